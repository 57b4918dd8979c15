"""Macro meshes of the workloads.

Each function returns (X, T): X float64 (nv, 3) vertex coordinates and T int32
(nt, 4) vertex ids per tetrahedron.  The vertex order inside a tetrahedron is
significant: uniform refinement cuts each octahedron along the line through
the midpoints of edges (x0,x2) and (x1,x3), so the order fixes the refined mesh.
"""
import functools
import itertools
import numpy as np


def unit_tet():
    """The unit reference tetrahedron (0,0,0),(1,0,0),(0,1,0),(0,0,1)."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    return X, np.array([[0, 1, 2, 3]], dtype=np.int32)


def regular_tet():
    """The regular tetrahedron of the paper's Fig. 5 (B)."""
    s = 1.0 / np.sqrt(2.0)
    X = np.array([[1, 0, -s], [-1, 0, -s], [0, 1, s], [0, -1, s]], dtype=np.float64)
    return X, np.array([[0, 1, 2, 3]], dtype=np.int32)


def flat_tet():
    """A flat macro tetrahedron with obtuse dihedral angles (its refined Laplacian
    has several positive off-diagonal stencil entries)."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.35, 0.35, 0.15]], dtype=np.float64)
    return X, np.array([[0, 1, 2, 3]], dtype=np.int32)


def _kuhn_tets(vid):
    """Six Kuhn tetrahedra of a cube whose corner (a,b,c) in {0,1}^3 has id
    vid(a,b,c), one per monotone path p0 = 0 -> p1 = e_p -> p2 = e_p+e_q ->
    p3 = 1, with vertices in the order (p2, p3, p0, p1).  That order refines
    exactly as the path order does (the octahedra are cut between the
    midpoints of p0p2 and p1p3 either way, so the refined cube is the
    Freudenthal lattice), and the two faces through the cube's diagonal p0p3,
    shared with the neighbouring tets, lie opposite the first and the last
    vertex."""
    tets = []
    for perm in itertools.permutations(range(3)):
        p = [0, 0, 0]
        path = [vid(*p)]
        for ax in perm:
            p[ax] = 1
            path.append(vid(*p))
        tets.append([path[2], path[3], path[0], path[1]])
    return tets


def kuhn_cube():
    """Unit cube split into 6 Kuhn tetrahedra sharing the main diagonal."""
    X = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)], dtype=np.float64)
    T = _kuhn_tets(lambda a, b, c: a + 2 * b + 4 * c)
    return X, np.array(T, dtype=np.int32)


def kuhn_cube_2x2x2():
    """Unit cube split into 2x2x2 sub-cubes, each into 6 Kuhn tetrahedra (48)."""
    X = np.array([[a / 2, b / 2, c / 2] for c in range(3) for b in range(3) for a in range(3)],
                 dtype=np.float64)
    T = []
    for oz, oy, ox in itertools.product(range(2), repeat=3):
        T += _kuhn_tets(lambda a, b, c: (ox + a) + 3 * (oy + b) + 9 * (oz + c))
    return X, np.array(T, dtype=np.int32)


def kuhn_box(nblocks, lo, hi):
    """The box [lo, hi] cut into nx x ny x nz equal blocks, each into its 6
    Kuhn tetrahedra (as kuhn_cube, along every block's lo -> hi diagonal, so
    the mesh is conforming and its uniform refinement is the Freudenthal
    triangulation of the fine grid)."""
    nx, ny, nz = nblocks
    g = [np.linspace(lo[d], hi[d], nb + 1) for d, nb in enumerate((nx, ny, nz))]
    X = np.array([[g[0][a], g[1][b], g[2][c]] for c in range(nz + 1) for b in range(ny + 1)
                  for a in range(nx + 1)], dtype=np.float64)
    vid = lambda a, b, c: a + (nx + 1) * (b + (ny + 1) * c)
    T = []
    for oz, oy, ox in itertools.product(range(nz), range(ny), range(nx)):
        T += _kuhn_tets(lambda a, b, c: vid(ox + a, oy + b, oz + c))
    return X, np.array(T, dtype=np.int32)


# reference domain of the paper's blending example (Sec. 7.4): radius
# (r1, r2) = (0.8, 1.0), angle (0, pi), height (0, z1), z1 = 4
CYLINDER_BOX = ((0.8, 0.0, 0.0), (1.0, np.pi, 4.0))


def cylinder_reference_box(nblocks=(1, 8, 10)):
    """The reference box of the half cylinder mantle of Sec. 7.4 in Kuhn
    blocks (default 80 blocks = 480 tets of 0.2 x 0.39 x 0.4)."""
    return kuhn_box(nblocks, *CYLINDER_BOX)


def orient_for_contiguous_faces(T, restarts=64, seed=0):
    """Vertex orders of the tets T (n, 4) that keep each tet's refinement and
    put as many shared faces as possible on contiguous runs of the slot
    layout in both tets holding them.  A tet refines the same in every order
    that keeps the vertex pairs {v0, v2} and {v1, v3} at positions {0, 2} and
    {1, 3} (the octahedra are cut between the midpoints of those two edges);
    among those orders, the faces opposite positions 0 and 3 are the
    contiguous ones.  Local search from seeded random starts; returns a new
    (n, 4) array."""
    T = np.asarray(T)
    faces = {}
    for t in range(len(T)):
        for q in range(4):
            faces.setdefault(tuple(sorted(np.delete(T[t], q))), []).append((t, int(T[t][q])))
    shared = [v for v in faces.values() if len(v) == 2]

    def options(tet):
        v0, v1, v2, v3 = (int(x) for x in tet)
        return [(a, dp, ap, d) for a, ap in ((v0, v2), (v2, v0)) for d, dp in ((v1, v3), (v3, v1))]

    def good(orders):
        return sum(1 for (t1, o1), (t2, o2) in shared
                   if o1 in (orders[t1][0], orders[t1][3]) and o2 in (orders[t2][0], orders[t2][3]))

    rng = np.random.default_rng(seed)
    best = (good([tuple(int(x) for x in t) for t in T]), [tuple(int(x) for x in t) for t in T])
    for _ in range(restarts):
        orders = [options(t)[rng.integers(4)] for t in T]
        score, improved = good(orders), True
        while improved:
            improved = False
            for t in range(len(T)):
                for o in options(T[t]):
                    old = orders[t]
                    orders[t] = o
                    s2 = good(orders)
                    if s2 > score:
                        score, improved = s2, True
                    else:
                        orders[t] = old
        if score > best[0]:
            best = (score, list(orders))
    return np.array(best[1], dtype=T.dtype)


def cube12_oriented_positive():
    """Unit cube split into 12 tetrahedra around one interior macro vertex at
    (0.5, 0.5, 0.5): every cube face is cut along a diagonal into two
    triangles (through (0,0,0) on the faces holding it, through (1,1,1) on
    the others) and each triangle is joined to the centre.  Tetrahedra are
    positively oriented, the centre last."""
    X = np.array([[a, b, c] for c in (0, 1) for b in (0, 1) for a in (0, 1)] + [[0.5, 0.5, 0.5]],
                 dtype=np.float64)
    vid = lambda a, b, c: a + 2 * b + 4 * c
    T = []
    for ax in range(3):
        for side in (0, 1):
            # the face's corners in cyclic order, starting at the diagonal's end
            o, p, q = ax, (ax + 1) % 3, (ax + 2) % 3
            def corner(u, v):
                c = [0, 0, 0]
                c[o], c[p], c[q] = side, u, v
                return vid(*c)
            if side == 0:
                ring = [corner(0, 0), corner(1, 0), corner(1, 1), corner(0, 1)]
            else:
                ring = [corner(1, 1), corner(0, 1), corner(0, 0), corner(1, 0)]
            for tri in ((ring[0], ring[1], ring[2]), (ring[0], ring[2], ring[3])):
                t = [tri[0], tri[1], tri[2], 8]
                e = X[t[1:]] - X[t[0]]
                if np.linalg.det(e) < 0:
                    t[1], t[2] = t[2], t[1]
                T.append(t)
    return X, np.array(T, dtype=np.int32)


def cube12():
    """cube12_oriented_positive's mesh with each tetrahedron in the vertex
    order of orient_for_contiguous_faces (the same refinement; 11 of the 18
    shared faces on contiguous slot runs in both tets, against 6)."""
    X, T = cube12_oriented_positive()
    return X, _cube12_orders(tuple(map(tuple, T)))


@functools.lru_cache(maxsize=None)
def _cube12_orders(T):
    return orient_for_contiguous_faces(np.array(T, dtype=np.int32))


MESHES = {
    "unit_tet": unit_tet,
    "regular_tet": regular_tet,
    "flat_tet": flat_tet,
    "kuhn_cube": kuhn_cube,
    "kuhn_cube_2x2x2": kuhn_cube_2x2x2,
    "cube12": cube12,
}


# ---------------------------------------------------------------- 2D macro meshes
# (X, T): X float64 (nv, 2), T int32 (nt, 3), every triangle counter-clockwise.

def _ccw(X, T):
    T = np.array(T, dtype=np.int32)
    for t in T:
        e = X[t[1:]] - X[t[0]]
        if e[0, 0] * e[1, 1] - e[0, 1] * e[1, 0] < 0:
            t[1], t[2] = t[2], t[1]
    return T


def obtuse_triangle():
    """One macro triangle with an obtuse angle (about 120 degrees) at (0.3, 0.25)."""
    X = np.array([[0.0, 0.0], [1.0, 0.0], [0.3, 0.25]])
    return X, _ccw(X, [[0, 1, 2]])


def square_right4():
    """Unit square cut into four right isosceles triangles at its centre: no
    obtuse angle, so the refined Laplacian is an M-matrix."""
    X = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0], [0.5, 0.5]])
    return X, _ccw(X, [[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]])


def square_nondelaunay8():
    """Unit square in eight triangles that is not Delaunay: the line y = 0.5
    from (0, 0.5) to (1, 0.5) is an interior macro edge whose two triangles
    have their obtuse angles (at (0.5, 0.4) and (0.5, 0.6)) facing it; each
    half of the square is a fan around one of those points."""
    X = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0], [0.0, 0.5], [1.0, 0.5],
                  [0.5, 0.4], [0.5, 0.6]])
    T = [[0, 1, 6], [1, 5, 6], [5, 4, 6], [4, 0, 6],
         [4, 5, 7], [5, 2, 7], [2, 3, 7], [3, 4, 7]]
    return X, _ccw(X, T)


MESHES2D = {
    "obtuse_triangle": obtuse_triangle,
    "square_right4": square_right4,
    "square_nondelaunay8": square_nondelaunay8,
}
