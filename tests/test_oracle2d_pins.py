"""Pins of the 2D oracle (oracle/oracle2d.py) against what the paper and the
mathematics fix: closed-form element matrices and lambda_min, exact
Galerkin matrices for constant k, Lemma 4.1 on a non-obtuse macro mesh, the
MA2 lemma (uniform positive definiteness after the modification) and the
pre-asymptotic loss of definiteness without it (Sec. 4.2), on a
non-Delaunay macro mesh of the unit square."""
import numpy as np
import pytest

from hhg_inputs import obtuse_triangle, square_right4, square_nondelaunay8, sigmoid_k, uniform_vector
from oracle import oracle2d as O2


def test_element_matrix_closed_forms():
    """Right triangle (0,0),(1,0),(0,1): A = 1/2 [[2,-1,-1],[-1,1,0],[-1,0,1]];
    equilateral triangle of side 1: A = [[2,-1,-1],...]/(2 sqrt 3), so both
    non-degenerate eigenvalues of A x = lambda B x equal 1/(2 sqrt 3); a
    triangle with an obtuse angle at vertex 2 has A[0,1] > 0."""
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [0.5, np.sqrt(3) / 2]])
    A, area = O2.element_matrices(xy, np.array([[0, 1, 2], [0, 1, 3]]))
    assert np.allclose(A[0], 0.5 * np.array([[2, -1, -1], [-1, 1, 0], [-1, 0, 1]]), atol=1e-15)
    assert np.allclose(area, [0.5, np.sqrt(3) / 4])
    assert np.allclose(A[1], O2._B / (2 * np.sqrt(3)), atol=1e-15)
    assert np.allclose(O2.lambda_min(A[1:]), [1 / (2 * np.sqrt(3))], atol=1e-14)
    X, T = obtuse_triangle()
    Ao, _ = O2.element_matrices(X, T.astype(np.int64))
    assert Ao[0, 0, 1] > 0 and Ao[0, 0, 2] < 0 and Ao[0, 1, 2] < 0
    assert np.abs(Ao.sum(axis=2)).max() <= 1e-15


@pytest.mark.parametrize("mesh_fn", [obtuse_triangle, square_nondelaunay8])
def test_constant_k_is_galerkin_without_modification(mesh_fn):
    X, T = mesh_fn()
    m = O2.Mesh2D(X, T, 3)
    k = np.full(m.n_nodes, 2.5)
    L = O2.assemble(m, np.ones(m.n_nodes), "nodal")
    mods, n_gray = O2.modification(m, k)
    assert n_gray > 0 and not mods
    for kind, mod in (("scaled", False), ("scaled", True), ("nodal", False)):
        M = O2.assemble(m, k, kind, mod)
        assert abs(M - 2.5 * L).max() <= 1e-13 * abs(L).max()


def test_refinement_counts_and_dirichlet():
    """8 n^2 elements; the six boundary macro edges carry 6 n Dirichlet nodes;
    Euler's formula for a triangulated disc gives 1 + 4 n^2 + 3 n nodes."""
    X, T = square_nondelaunay8()
    for lv in (0, 1, 3):
        m = O2.Mesh2D(X, T, lv)
        n = 2 ** lv
        assert m.conn.shape[0] == 8 * n * n
        assert m.dirichlet.sum() == 6 * n
        assert m.n_nodes == 1 + 4 * n * n + 3 * n
        b = m.xy[m.dirichlet]
        assert np.all((np.isclose(b, 0) | np.isclose(b, 1)).any(axis=1))


def test_lemma_4_1_non_obtuse_mesh_is_semidefinite():
    """No obtuse macro angle: the Laplacian is an M-matrix and the scaled form
    is positive semi-definite for any positive k, however steep."""
    X, T = square_right4()
    for lv in (1, 2, 3):
        m = O2.Mesh2D(X, T, lv)
        L = O2.assemble(m, np.ones(m.n_nodes), "nodal").toarray()
        off = L - np.diag(np.diag(L))
        assert off.max() <= 1e-14
        for eta in (1.0, 1000.0):
            A = O2.reduced(m, O2.assemble(m, sigmoid_k(m.xy, eta), "scaled")).toarray()
            assert np.linalg.eigvalsh(A)[0] >= -1e-10 * np.abs(A).max()
        assert not O2.modification(m, sigmoid_k(m.xy, 1000.0))[1]


@pytest.mark.parametrize("eta", [1.0, 10.0, 100.0, 1000.0])
def test_ma2_restores_definiteness(eta):
    """Sec. 4.1 lemma: with (MA2) the form is positive definite on the
    unknowns at every level; every replaced factor lies strictly between
    k_{e;min} and k_e; nodal integration is positive definite.  Sec. 4.2:
    without it, a steep k (eta >= 10) gives negative eigenvalues in the
    pre-asymptotic regime."""
    X, T = square_nondelaunay8()
    negative = []
    for lv in range(4):
        m = O2.Mesh2D(X, T, lv)
        k = sigmoid_k(m.xy, eta)
        ev = {}
        for kind, mod in (("scaled", False), ("scaled", True), ("nodal", False)):
            A = O2.reduced(m, O2.assemble(m, k, kind, mod)).toarray()
            assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
            ev[(kind, mod)] = np.linalg.eigvalsh(A)[0]
        assert ev[("scaled", True)] > 0 and ev[("nodal", False)] > 0
        negative.append(ev[("scaled", False)] < 0)
        mods, _ = O2.modification(m, k)
        for (Tm, lo, hi), km in mods.items():
            assert km < (k[lo] + k[hi]) / 2
    assert any(negative) == (eta >= 10.0)


def test_scaled_and_nodal_agree_asymptotically():
    """Lemma 3.1 setting: for smooth k the scaled and nodal rows of nodes
    inside the macro triangles differ by O(h^2) relative on smooth functions."""
    X, T = square_nondelaunay8()
    gaps = []
    for lv in (3, 4, 5):
        m = O2.Mesh2D(X, T, lv)
        k = 1.0 + 0.5 * np.sin(2 * np.pi * m.xy[:, 0]) * np.cos(np.pi * m.xy[:, 1])
        u = np.sin(np.pi * m.xy[:, 0]) * np.sin(np.pi * m.xy[:, 1])
        S = O2.apply(m, O2.assemble(m, k, "scaled"), u)
        N = O2.apply(m, O2.assemble(m, k, "nodal"), u)
        inner = (m.prim_dim == 2) & ~m.dirichlet
        gaps.append(np.abs(S - N)[inner].max() / np.abs(N[inner]).max())
    assert gaps[0] > gaps[1] > gaps[2] and gaps[1] / gaps[2] > 3.0, gaps


@pytest.mark.parametrize("kind", ["scaled", "nodal"])
def test_l2_rate_on_a_manufactured_solution(kind):
    """Lemma 3.1 (as in the 2D study of Sec. 7.1): with u* = sin(pi x) sin(pi y),
    k = 2 + sin(2 pi x) sin(2 pi y) and b = M f, the discrete L2 error of
    I_h u* - u_h converges at order 2 on the non-Delaunay square."""
    X, T = square_nondelaunay8()
    pi = np.pi
    errs = []
    for lv in (3, 4, 5, 6):
        m = O2.Mesh2D(X, T, lv)
        x, y = m.xy[:, 0], m.xy[:, 1]
        us = np.sin(pi * x) * np.sin(pi * y)
        k = 2 + np.sin(2 * pi * x) * np.sin(2 * pi * y)
        kx, ky = 2 * pi * np.cos(2 * pi * x) * np.sin(2 * pi * y), 2 * pi * np.sin(2 * pi * x) * np.cos(2 * pi * y)
        ux, uy = pi * np.cos(pi * x) * np.sin(pi * y), pi * np.sin(pi * x) * np.cos(pi * y)
        f = -(kx * ux + ky * uy) + 2 * pi * pi * k * us
        Mm = O2.assemble_mass(m)
        uh = O2.solve(m, O2.assemble(m, k, kind, kind == "scaled"), Mm @ f)
        e = us - uh
        e[m.dirichlet] = 0.0
        errs.append(np.sqrt(e @ (Mm @ e)))
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(eoc[1:] > 1.85) and abs(eoc[-1] - 2.0) < 0.1, eoc


def test_scaled_quadratic_form_is_the_edge_sum():
    """The identity in the proof of Lemma 4.1: for the unmodified scaled form,
    v^T A v = -1/4 sum_{i,j} (k_i + k_j) (v_i - v_j)^2 (A_hat)_{ij} with A_hat
    the constant-coefficient (k = 1) matrix -- evaluated here pair by pair
    from A_hat, independently of the element-wise assembly with zero row sums."""
    X, T = square_nondelaunay8()
    m = O2.Mesh2D(X, T, 2)
    k = sigmoid_k(m.xy, 100.0)
    A = O2.assemble(m, k, "scaled").toarray()
    Ahat = O2.assemble(m, np.ones(m.n_nodes), "nodal").tocoo()
    rng = np.random.default_rng(3)
    for _ in range(3):
        v = rng.uniform(-1, 1, m.n_nodes)
        i, j, a = Ahat.row, Ahat.col, Ahat.data
        edge = -0.25 * np.sum((k[i] + k[j]) * (v[i] - v[j]) ** 2 * a)
        assert abs(v @ A @ v - edge) <= 1e-12 * abs(edge)
