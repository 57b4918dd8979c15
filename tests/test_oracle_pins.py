"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: printed
values (Fig. 5), the paper's lemmas (exactness for constant k, equality of the
scaled and nodal forms for affine k, O(h^2) consistency, positivity, optimal
convergence rates), literal evaluation of the defining formulas, closed forms
(Chebyshev polynomials, exact quadrature, linear reproduction).
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from hhg_inputs import (unit_tet, regular_tet, flat_tet, kuhn_cube, kuhn_cube_2x2x2, cube12, smooth_k,
                        affine_k, sigmoid_k, manufactured_u, uniform_vector, manufactured_f,
                        lognormal_params, lognormal_k, tensor_K, tensor_fields)
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lattice_offset(mesh, T, c, j):
    """tet-local lattice offset of node j relative to node c in macro tet T."""
    X = mesh.X[mesh.T[T]]
    E = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
    n = 2 ** mesh.level
    return tuple(np.rint(np.linalg.solve(E, mesh.xyz[j] - mesh.xyz[c]) * n).astype(int))


def _two_sig(x):
    return float(f"{x:.1e}")


def test_fig5_reference_stencils_match_printed_values():
    """Fig. 5: level-2 interior stencils of the unit and the regular tetrahedron."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fig5_stencils.txt"))
            if l.strip() and not l.startswith("#")]
    for panel, fn in (("A", unit_tet), ("B", regular_tet)):
        X, T = fn()
        m = O.Mesh(X, T, 2)
        A = O.assemble(m, np.ones(m.n_nodes)).toarray()
        c = m.unknowns[0]               # the single interior node at level 2
        got = {}
        for j in np.flatnonzero(A[c]):
            got[_lattice_offset(m, 0, c, j)] = A[c, j]
        want = {(int(r[1]), int(r[2]), int(r[3])): float(r[4]) for r in rows if r[0] == panel}
        assert set(got) == set(want), panel
        for d, v in want.items():
            assert _two_sig(got[d]) == pytest.approx(v, rel=1e-12), (panel, d, got[d], v)


@pytest.mark.parametrize("mesh_fn,level", [(unit_tet, 3), (kuhn_cube, 2), (kuhn_cube_2x2x2, 2)])
def test_constant_k_is_exact(mesh_fn, level):
    """k constant: scaled = nodal = k * Laplacian (Sec. 2.1: a_h = a for constant k)."""
    X, T = mesh_fn()
    m = O.Mesh(X, T, level)
    lap = O.assemble(m, np.ones(m.n_nodes), "nodal").toarray()
    k = np.full(m.n_nodes, 2.75)
    As = O.assemble(m, k, "scaled").toarray()
    An = O.assemble(m, k, "nodal").toarray()
    s = np.abs(lap).max()
    assert np.abs(As - 2.75 * lap).max() <= 1e-14 * s
    assert np.abs(An - 2.75 * lap).max() <= 1e-14 * s


@pytest.mark.parametrize("mesh_fn,level", [(unit_tet, 3), (regular_tet, 3), (kuhn_cube_2x2x2, 2)])
def test_zero_row_sum_and_symmetry(mesh_fn, level):
    """Row sums vanish and the matrices are symmetric (Sec. 2.2, eq. (zerosum), Lemma 3.2)."""
    X, T = mesh_fn()
    m = O.Mesh(X, T, level)
    k = smooth_k(m.xyz) + m.xyz[:, 0]
    for kind in ("scaled", "nodal"):
        A = O.assemble(m, k, kind)
        s = abs(A).max()
        assert np.abs(A @ np.ones(m.n_nodes)).max() <= 1e-14 * s * 15
        assert abs(A - A.T).max() <= 1e-15 * s * 4


@pytest.mark.parametrize("mesh_fn,level", [(unit_tet, 2), (kuhn_cube, 1), (regular_tet, 2)])
def test_brute_force_definitions(mesh_fn, level):
    """eq. (discrete) and eq. (standardfe) evaluated literally over node pairs /
    quadrature points equal the element-loop assembly (Lemma 3.2)."""
    X, T = mesh_fn()
    m = O.Mesh(X, T, level)
    k = 1.0 + m.xyz[:, 0] ** 2 + np.sin(3 * m.xyz[:, 1]) ** 2 + 0.3 * m.xyz[:, 2]
    As = O.assemble(m, k, "scaled").toarray()
    Bs = O.brute_force_scaled(m, k)
    assert np.abs(As - Bs).max() <= 1e-14 * np.abs(As).max()
    An = O.assemble(m, k, "nodal").toarray()
    Bn = O.brute_force_nodal(m, k)
    assert np.abs(An - Bn).max() <= 1e-14 * np.abs(An).max()


def _tet_interior_mask(m):
    """Nodes strictly inside a macro tet: the last block of the canonical order."""
    n = 2 ** m.level
    per = (n - 1) * (n - 2) * (n - 3) // 6
    mask = np.zeros(m.n_nodes, dtype=bool)
    mask[m.n_nodes - per * m.T.shape[0]:] = True
    return mask


@pytest.mark.parametrize("mesh_fn,level", [(unit_tet, 3), (unit_tet, 4), (regular_tet, 3), (kuhn_cube, 3)])
def test_affine_k_scaled_equals_nodal_on_volume_rows(mesh_fn, level):
    """k affine: the point-reflection argument of Lemma 3.3 (and Lemma 5.1) makes
    the scaled and nodal rows of macro-interior nodes identical."""
    X, T = mesh_fn()
    m = O.Mesh(X, T, level)
    k = affine_k(m.xyz)
    As = O.assemble(m, k, "scaled")
    An = O.assemble(m, k, "nodal")
    v = _tet_interior_mask(m)
    D = (As - An).tocsr()[v]
    assert abs(D).max() <= 1e-14 * abs(An).max()


def test_consistency_gap_is_second_order():
    """A3 / Lemma 3.3: for smooth k the scaled-vs-nodal entry gap on macro-interior
    rows shrinks like h^2 relative to the entries."""
    X, T = unit_tet()
    gaps = []
    for L in (4, 5, 6):
        m = O.Mesh(X, T, L)
        k = smooth_k(m.xyz)
        As = O.assemble(m, k, "scaled")
        An = O.assemble(m, k, "nodal")
        v = _tet_interior_mask(m)
        gaps.append(abs((As - An).tocsr()[v]).max() / abs(An.tocsr()[v]).max())
    r1, r2 = gaps[0] / gaps[1], gaps[1] / gaps[2]
    assert 3.0 < r1 < 5.0 and 3.5 < r2 < 4.5, gaps


def test_m_matrix_mesh_gives_positive_operator():
    """Lemma 4.1: Kuhn macro tets give an M-matrix Laplacian, so the scaled form
    stays positive (definite on the unknowns) even for a steep coefficient."""
    X, T = kuhn_cube()
    m = O.Mesh(X, T, 2)
    k = sigmoid_k(m.xyz, eta=1000.0)
    op = O.make_operator(m, k, "scaled")
    assert np.linalg.eigvalsh(op.A.toarray()).min() > 0
    mods, info = O.modification_factors(m, k)
    assert info["n_candidates"] == 0 and not mods


def test_modification_properties():
    """Sec. 4.1 read for 3D: no trigger for constant k; k_emin < k_mod < k_e on
    triggered edges; the modification restores positivity where the plain
    scaled matrix of an M-matrix-free mesh is indefinite."""
    X, T = unit_tet()
    m = O.Mesh(X, T, 3)
    mods, info = O.modification_factors(m, np.full(m.n_nodes, 3.0))
    assert info["n_candidates"] > 0 and not mods
    # lambda_min^T / a_plus is a property of the macro tet, independent of the level
    ratios = []
    for L in (2, 3):
        mm = O.Mesh(X, T, L)
        _, inf = O.modification_factors(mm, np.ones(mm.n_nodes))
        ratios.append(inf["lam_T"][0] / inf["a_plus"].max())
    assert ratios[0] == pytest.approx(ratios[1], rel=1e-12)
    found_indefinite = False
    X, T = flat_tet()
    for L in (2, 3):
        mm = O.Mesh(X, T, L)
        if len(mm.unknowns) == 0:
            continue
        for eta in (100.0, 1000.0):
            k = sigmoid_k(mm.xyz, eta)
            mods, inf = O.modification_factors(mm, k)
            if inf["n_triggered"]:
                assert np.all(inf["k_emin"] < inf["k_mod"]) and np.all(inf["k_mod"] < inf["k_e"])
            plain = O.make_operator(mm, k, "scaled").A.toarray()
            fixed = O.make_operator(mm, k, "scaled", modification=True).A.toarray()
            if np.linalg.eigvalsh(plain).min() < 0:
                found_indefinite = True
            assert np.linalg.eigvalsh(fixed).min() > 0, (L, eta)
    assert found_indefinite, "the steep coefficient should break positivity somewhere"


def test_prolongation_reproduces_affine_functions():
    for fn, L in ((unit_tet, 2), (kuhn_cube_2x2x2, 1)):
        X, T = fn()
        mc, mf = O.Mesh(X, T, L), O.Mesh(X, T, L + 1)
        P = O.prolongation(mc, mf)
        g = lambda x: 0.3 + 2 * x[:, 0] - x[:, 1] + 4 * x[:, 2]
        assert np.abs(P @ g(mc.xyz) - g(mf.xyz)).max() < 1e-13
        c2f = O.coarse_to_fine(mc, mf)
        assert np.abs(mf.xyz[c2f] - mc.xyz).max() < 1e-15


def test_quadrature_and_mass_are_exact():
    """Stroud conical rule integrates monomials of degree <= 5 exactly on the unit
    tet (int x^a y^b z^c = a! b! c! / (a+b+c+3)!); the mass matrix sums to |Omega|."""
    bary, w = O._conical_rule(4)
    pts = bary[:, 1:]
    for a, b, c in [(0, 0, 0), (1, 2, 2), (5, 0, 0), (2, 1, 2), (0, 3, 2)]:
        exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
        assert np.sum(w * pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c) == pytest.approx(exact, rel=1e-13)
    X, T = kuhn_cube()
    m = O.Mesh(X, T, 2)
    M = O.assemble_mass(m)
    assert M.sum() == pytest.approx(1.0, rel=1e-14)


def test_rows_one_by_one_match_full_assembly():
    for fn, L in ((unit_tet, 3), (kuhn_cube_2x2x2, 2)):
        X, T = fn()
        m = O.Mesh(X, T, L)
        k = smooth_k(m.xyz) + 0.5
        for kind in ("scaled", "nodal"):
            A = O.assemble(m, k, kind).tocsr()
            nodes = np.random.default_rng(0).choice(m.n_nodes, 25, replace=False)
            for p, (c, v) in zip(nodes, O.rows(m, k, nodes, kind)):
                ref = A[p].toarray().ravel()
                got = np.zeros(m.n_nodes)
                got[c] = v
                assert np.abs(ref - got).max() <= 1e-14 * np.abs(ref).max()


def test_chebyshev_matches_closed_form():
    """On D^{-1}A with known spectrum the error is multiplied by
    T_s((theta - lam)/delta) / T_s(theta/delta) per eigen-component."""
    class Diag:
        pass
    lam = np.linspace(0.05, 2.0, 40)
    import scipy.sparse as sp
    from types import SimpleNamespace
    mesh = SimpleNamespace(n_nodes=40, unknowns=np.arange(40), dirichlet=np.zeros(40, bool))
    op = SimpleNamespace(mesh=mesh, A=sp.diags(lam).tocsr(), diag=np.ones(40))
    op.apply = lambda x: op.A @ x
    op.residual = lambda f, x: f - op.A @ x
    e0 = np.ones(40)
    lmax = 2.0
    for s in (1, 2, 3, 4):
        u = O.chebyshev(op, np.zeros(40), e0, s, lmax)
        a, b = 0.1 * lmax, 1.0 * lmax
        th, de = (a + b) / 2, (b - a) / 2
        Ts = lambda x: np.cosh(s * np.arccosh(x)) if np.all(np.abs(x) >= 1) else np.cos(s * np.arccos(np.clip(x, -1, 1)))
        Tx = np.array([np.polynomial.chebyshev.chebval((th - l) / de, [0] * s + [1]) for l in lam])
        ref = Tx / np.polynomial.chebyshev.chebval(th / de, [0] * s + [1])
        assert np.abs(u - ref).max() < 1e-12


def test_jacobi_fixed_point_and_multigrid_solution():
    X, T = kuhn_cube()
    mg = O.Multigrid(X, T, 4, 2, kfun=smooth_k)
    m = mg.meshes[4]
    op = mg.ops[4]
    f = np.zeros(m.n_nodes)
    f[m.unknowns] = np.random.default_rng(3).uniform(-1, 1, len(m.unknowns))
    ref = np.zeros(m.n_nodes)
    ref[m.unknowns] = spla.spsolve(op.A.tocsc(), f[m.unknowns])
    u, hist = mg.solve(f, tol=1e-10)
    assert all(h2 < h1 for h1, h2 in zip(hist, hist[1:]))
    assert np.abs(u - ref).max() <= 1e-8 * np.abs(ref).max()
    rho = (hist[-1] / hist[1]) ** (1.0 / (len(hist) - 2))
    assert rho < 0.35
    # Gershgorin bound of D^-1 A for the 7-point-type Kuhn stencil is exactly 2
    assert O.gershgorin_lambda(op) == pytest.approx(2.0, rel=1e-12) or O.gershgorin_lambda(op) <= 2.0 + 1e-12
    # Jacobi keeps the exact solution fixed
    uj = O.jacobi(op, f, ref, 3)
    assert np.abs(uj - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.slow
def test_convergence_rates_manufactured_solution():
    """Lemma 3.1: O(h^2) in L2 and O(h) in H1 for the scaled form (and the
    nodal form), 6-tet Kuhn cube, u = sin sin sin, k = smooth_k, b = M I_h f."""
    X, T = kuhn_cube()
    res = {"scaled": [], "nodal": []}
    grad = lambda x: np.pi * np.stack([
        np.cos(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]) * np.sin(np.pi * x[:, 2]),
        np.sin(np.pi * x[:, 0]) * np.cos(np.pi * x[:, 1]) * np.sin(np.pi * x[:, 2]),
        np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]) * np.cos(np.pi * x[:, 2])], axis=1)
    for L in (2, 3, 4, 5):
        m = O.Mesh(X, T, L)
        b = O.assemble_mass(m) @ manufactured_f(m.xyz)
        k = smooth_k(m.xyz)
        for kind in res:
            op = O.make_operator(m, k, kind)
            uh = np.zeros(m.n_nodes)
            uh[m.unknowns] = spla.spsolve(op.A.tocsc(), b[m.unknowns])
            res[kind].append(O.errors(m, uh, manufactured_u, grad))
    for kind, errs in res.items():
        eoc_l2 = [np.log2(a["L2"] / b["L2"]) for a, b in zip(errs, errs[1:])]
        eoc_h1 = [np.log2(a["H1"] / b["H1"]) for a, b in zip(errs, errs[1:])]
        eoc_nd = [np.log2(a["nodal_L2"] / b["nodal_L2"]) for a, b in zip(errs, errs[1:])]
        assert abs(eoc_l2[-1] - 2.0) < 0.15, (kind, eoc_l2)
        assert abs(eoc_nd[-1] - 2.0) < 0.15, (kind, eoc_nd)
        assert abs(eoc_h1[-1] - 1.0) < 0.1, (kind, eoc_h1)
    ratio = res["scaled"][-1]["nodal_L2"] / res["nodal"][-1]["nodal_L2"]
    assert 0.3 < ratio < 3.0


def test_canonical_order_convention():
    """Canonical numbering: macro vertices first, then edge, face and tet-interior nodes."""
    X, T = unit_tet()
    m = O.Mesh(X, T, 2)
    assert np.allclose(m.xyz[:4], X)
    # edge (0,1): nodes at 1/4, 2/4, 3/4 along x
    assert np.allclose(m.xyz[4:7], [[0.25, 0, 0], [0.5, 0, 0], [0.75, 0, 0]])
    # the only interior node of the level-2 tet is last
    assert np.allclose(m.xyz[-1], [0.25, 0.25, 0.25]) and m.unknowns.tolist() == [m.n_nodes - 1]
    X, T = kuhn_cube_2x2x2()
    m = O.Mesh(X, T, 1)
    assert len(m.unknowns) == 27 and m.n_nodes == 125


def test_primitive_dims_match_closed_form_counts():
    """Sec. 5 node sets of the 12-tet cube (9 vertices, 26 edges, 30 faces):
    per level n = 2^l, (n-1) nodes per edge, (n-1)(n-2)/2 per face,
    (n-1)(n-2)(n-3)/6 per tet interior."""
    X, T = cube12()
    for level in (2, 3):
        n = 2 ** level
        m = O.Mesh(X, T, level)
        counts = np.bincount(O.primitive_dims(m), minlength=4).tolist()
        assert counts == [9, 26 * (n - 1), 30 * (n - 1) * (n - 2) // 2, 12 * (n - 1) * (n - 2) * (n - 3) // 6]
        # the interior of the cube: 1 vertex, 8 edges, 18 faces, 12 tets
        d = O.primitive_dims(m)[m.unknowns]
        assert np.bincount(d, minlength=4).tolist() == [1, 8 * (n - 1), 18 * (n - 1) * (n - 2) // 2,
                                                        12 * (n - 1) * (n - 2) * (n - 3) // 6]


@pytest.mark.parametrize("level", [2, 3])
def test_primitive_mix_reproduces_affine_solutions(level):
    """Lemma 5.1 on the 12-tet unit cube with u = -7x+y+3z, k = 2x+3y+5z+1
    (the paper's example; f = -div(k grad u) = -4): the nodal-integration
    operator and a_{h;I} with I = W or W_V u W_E reproduce u to rounding, both
    as a solve with the exact Dirichlet data and in the operator form
    a_{h;I}(u, phi_i) = a~_h(u, phi_i) on the interior rows; stencil scaling
    alone and the mixes without edges (or without vertices) do not."""
    X, T = cube12()
    m = O.Mesh(X, T, level)
    x = m.xyz
    k = affine_k(x)
    u = -7.0 * x[:, 0] + x[:, 1] + 3.0 * x[:, 2]
    b = O.assemble_mass(m) @ np.full(m.n_nodes, -4.0)
    I, D = m.unknowns, np.flatnonzero(m.dirichlet)
    N = O.assemble(m, k, "nodal")
    scale = np.abs((N @ u)[I]).max()

    def err(A):
        A = A.tocsr()
        uh = u.copy()
        uh[I] = spla.spsolve(A[I][:, I].tocsc(), b[I] - A[I][:, D] @ u[D])
        return np.sqrt(m.h ** 3 * np.sum((uh - u) ** 2))

    assert err(N) < 1e-13
    for dims in ((0, 1, 2), (0, 1)):
        A = O.assemble_mixed(m, k, dims)
        assert err(A) < 1e-13, dims
        assert np.abs(((A - N) @ u)[I]).max() <= 1e-10 * scale, dims
    for dims in ((), (0,), (0, 2), (1,), (1, 2)):
        A = O.assemble_mixed(m, k, dims) if dims else O.assemble(m, k, "scaled")
        assert err(A) > 1e-5, dims
        assert np.abs(((A - N) @ u)[I]).max() > 1e-2 * scale, dims


@pytest.mark.parametrize("mesh_fn", [cube12, kuhn_cube])
def test_tensor_constant_K_is_exact_galerkin(mesh_fn):
    """Sec. 2.1 eq. (integral) with constant K: every component's coefficient
    is constant, so scaling and nodal integration both give the exact
    Galerkin matrix of grad v . K grad w (|t| G K G^T); this also pins the
    six-component decomposition of K."""
    X, T = mesh_fn()
    m = O.Mesh(X, T, 2)
    K = np.array([[2.0, 0.3, -0.2], [0.3, 1.5, 0.4], [-0.2, 0.4, 1.2]])
    K6 = tensor_fields(np.broadcast_to(K, (m.n_nodes, 3, 3)))
    G = O.assemble_galerkin_constant_tensor(m, K)
    for kind in ("scaled", "nodal"):
        A = O.assemble_tensor(m, K6, kind)
        assert abs(A - G).max() <= 1e-13 * abs(G).max(), kind


def test_tensor_scalar_K_is_the_scalar_operator():
    """K = k I: the tensor form reduces to -div(k grad u) (M = 1, Sec. 2.1)."""
    X, T = cube12()
    m = O.Mesh(X, T, 3)
    k = smooth_k(m.xyz)
    K6 = tensor_fields(k[:, None, None] * np.eye(3)[None])
    for kind in ("scaled", "nodal"):
        A, S = O.assemble_tensor(m, K6, kind), O.assemble(m, k, kind)
        assert abs(A - S).max() <= 1e-13 * abs(S).max(), kind


def test_tensor_operator_symmetric_with_zero_row_sums():
    """Variable SPD K: the scaled tensor matrix is symmetric (Lemma 3.2 per
    component), its rows sum to zero and it is positive definite on the
    unknowns; on macro-interior rows scaling and nodal integration differ by
    O(h^2) for smooth u (ratio -> 4 per level)."""
    X, T = kuhn_cube()
    gaps = []
    for level in (3, 4, 5):
        m = O.Mesh(X, T, level)
        K6 = tensor_fields(tensor_K(m.xyz))
        A = O.assemble_tensor(m, K6)
        assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
        assert np.abs(A @ np.ones(m.n_nodes)).max() <= 1e-12 * abs(A).max()
        if level == 3:
            Au = A[m.unknowns][:, m.unknowns].toarray()
            assert np.linalg.eigvalsh(Au).min() > 0
        N = O.assemble_tensor(m, K6, "nodal")
        u = manufactured_u(m.xyz)
        inner = np.flatnonzero((O.primitive_dims(m) == 3) & ~m.dirichlet)
        gaps.append(np.abs(((A - N) @ u)[inner]).max() / np.abs((N @ u)[inner]).max())
    assert gaps[0] > gaps[1] > gaps[2] and gaps[1] / gaps[2] > 3.3, gaps


@pytest.mark.parametrize("kind", ["scaled", "nodal"])
def test_tensor_rows_from_incident_elements_match_assembly(kind):
    """The row-restricted evaluation (for sizes the assembly cannot reach)
    agrees with the assembled matrix on macro-vertex, edge, face, interior
    and Dirichlet nodes."""
    X, T = cube12()
    m = O.Mesh(X, T, 3)
    K6 = tensor_fields(tensor_K(m.xyz))
    u = uniform_vector(m.n_nodes, seed=5)
    u[m.dirichlet] = 0.0
    full = O.make_tensor_operator(m, K6, kind).apply(u)
    dims = O.primitive_dims(m)
    rng = np.random.default_rng(2)
    nodes = np.concatenate([rng.choice(np.flatnonzero(dims == d), 4, replace=False) for d in range(4)]
                           + [np.flatnonzero(m.dirichlet)[:3]])
    got = O.apply_tensor_rows(m, lambda x: tensor_fields(tensor_K(x)), u, nodes, kind)
    assert np.abs(got - full[nodes]).max() <= 1e-13 * np.abs(full).max()


def _node_at(mesh, lat):
    """Canonical index of the unit-tet node with lattice coordinates lat."""
    x = np.asarray(lat, dtype=np.float64) / 2 ** mesh.level
    d = np.abs(mesh.xyz - x).max(axis=1)
    j = int(np.argmin(d))
    assert d[j] < 1e-14
    return j


def test_modification_ratio_and_patch_enumerated_by_hand():
    """Sec. 4.1 read for 3D.  (i) lambda_min^T / a_plus = 0.1464 on the unit
    tet at every level: the corner children are the parent scaled by h (their
    matrix |t| G G^T = h/6 [[3,-1,-1,-1],[-1,1,0,0],[-1,0,1,0],[-1,0,0,1]] has
    lambda_2/4 = h/24), the octahedral children give the minimum 0.02440 h,
    and the largest positive element entry is h/6.  (ii) k_emin of one edge
    is the minimum over exactly the 13 edges of the four elements around it
    (the edge, its 4 links to each end, the 4-cycle of link vertices):
    neither the link cycle's diagonals nor edges elsewhere around the end
    points may enter."""
    X, T = unit_tet()
    for L in (2, 3, 4):
        m = O.Mesh(X, T, L)
        _, info = O.modification_factors(m, np.ones(m.n_nodes))
        h = 2.0 ** -L
        assert info["a_plus"].max() == pytest.approx(h / 6, rel=1e-12)
        assert info["lam_T"][0] / info["a_plus"].max() == pytest.approx(0.1464, abs=5e-5)
    ratio = info["lam_T"][0] / info["a_plus"].max()
    m = O.Mesh(X, T, 3)
    i = np.array([2, 3, 1])
    d = np.array([1, -1, 1])                        # the gray Bey diagonal
    j = i + d
    la, lb, lc, le = (i + np.array(o) for o in ((0, -1, 1), (0, 0, 1), (1, -1, 0), (1, 0, 0)))
    o1, o2 = i + np.array([-1, 0, 0]), i + np.array([0, -1, 0])   # neighbours of i off the patch
    k = np.ones(m.n_nodes)
    for p, v in ((i, 100.0), (j, 100.0), (la, 0.01), (le, 0.01), (o1, 1e-3), (o2, 1e-3)):
        k[_node_at(m, p)] = v
    # patch edges: i-j, i-links, j-links and the cycle a-b-e-c-a; the smallest
    # average is on a cycle edge with one end at a or e: (0.01 + 1)/2.  The
    # diagonal a-e would give 0.01, the edge o1-o2 near i would give 1e-3.
    mods, info = O.modification_factors(m, k)
    a, b = sorted((_node_at(m, i), _node_at(m, j)))
    assert (0, a, b) in mods
    assert mods[(0, a, b)] == pytest.approx(0.505 * (1.0 + ratio), rel=1e-12)


def test_mass_matrix_is_the_exact_l2_product():
    """u'Mv equals the integral of u_h v_h (P1 interpolants), computed by the
    degree-5 quadrature per element; a lumped or mis-scaled mass fails."""
    for fn, L in ((unit_tet, 2), (regular_tet, 2), (kuhn_cube, 1)):
        X, T = fn()
        m = O.Mesh(X, T, L)
        M = O.assemble_mass(m)
        rng = np.random.default_rng(3)
        u = rng.uniform(-1, 1, m.n_nodes)
        zero = lambda x: np.zeros(len(x))
        gzero = lambda x: np.zeros((len(x), 3))
        quad = O.errors(m, u, zero, gzero)["L2"] ** 2
        assert u @ (M @ u) == pytest.approx(quad, rel=1e-12)
        # polarisation: the bilinear form, not just the quadratic one
        v = rng.uniform(-1, 1, m.n_nodes)
        q2 = O.errors(m, u + v, zero, gzero)["L2"] ** 2
        q3 = O.errors(m, u - v, zero, gzero)["L2"] ** 2
        assert u @ (M @ v) == pytest.approx((q2 - q3) / 4, rel=1e-10, abs=1e-14)


def test_threaded_csr_product_equals_the_assembled_operator():
    """The C CSR product used to time the oracle gives op.apply's result
    exactly (same per-row summation order) for 1 and several threads, and the
    dense product up to rounding."""
    X, T = kuhn_cube_2x2x2()
    m = O.Mesh(X, T, 2)
    k = lognormal_k(m.xyz, lognormal_params(1, 1.0, 0.1))
    op = O.make_operator(m, k, "scaled", modification=True)
    x = uniform_vector(m.n_nodes, seed=7)
    x[m.dirichlet] = 0.0
    ref = op.apply(x)
    for th in (1, 3):
        assert np.array_equal(O.spmv_threaded(op, x, th), ref)
    dense = np.zeros(m.n_nodes)
    dense[m.unknowns] = op.A.toarray() @ x[m.unknowns]
    assert np.abs(ref - dense).max() <= 1e-14 * np.abs(dense).max()
    t = O.spmv_bench(op, 2, warm=1, reps=3)
    assert t.shape == (3,) and np.all(t > 0)


def test_kuhn_cube_mass_rhs_matches_the_oracle_mass_matrix():
    """The grid-stencil rhs b = M I_h f used for the 6-tet cube at large levels
    equals the oracle's assembled consistent mass matrix times f on every
    unknown (the refined Kuhn cube is the Freudenthal triangulation)."""
    from hhg_inputs import kuhn_cube_mass_rhs
    X, T = kuhn_cube()
    for L in (2, 3):
        m = O.Mesh(X, T, L)
        want = O.assemble_mass(m) @ manufactured_f(m.xyz)
        got = kuhn_cube_mass_rhs(m.xyz, L, manufactured_f)
        u = m.unknowns
        assert np.abs(got[u] - want[u]).max() <= 1e-13 * np.abs(want[u]).max()


def test_geometric_coarse_coefficients():
    """k_c = exp(sum_f P_fc log k_f / sum_f P_fc): constant k stays constant;
    for log k affine the average equals k at every macro-tet interior coarse
    node (its support, the node and the 14 edge midpoints, is point
    symmetric); at one boundary node, the support enumerated from the coarse
    edges of the refined mesh (element vertex pairs) gives the same value."""
    X, T = kuhn_cube_2x2x2()
    mc, mf = O.Mesh(X, T, 2), O.Mesh(X, T, 3)
    P = O.prolongation(mc, mf)
    assert np.allclose(O.geometric_coarse_k(P, np.full(mf.n_nodes, 2.5)), 2.5, rtol=1e-15, atol=0)
    g = lambda x: 0.3 + 0.7 * x[:, 0] - 1.1 * x[:, 1] + 0.4 * x[:, 2]
    kc = O.geometric_coarse_k(P, np.exp(g(mf.xyz)))
    interior = O.primitive_dims(mc) == 3
    assert interior.sum() > 0
    assert np.abs(kc[interior] / np.exp(g(mc.xyz[interior])) - 1).max() < 1e-13
    # one node on the domain boundary and one on an interior macro vertex
    kf = lognormal_k(mf.xyz, lognormal_params(2, 1.5, 0.05))
    kc = O.geometric_coarse_k(P, kf)
    conn, _ = mc.elements()
    c2f = O.coarse_to_fine(mc, mf)
    for c in (int(np.flatnonzero(mc.dirichlet)[5]), int(np.argmin(np.abs(mc.xyz - 0.5).sum(axis=1)))):
        nbrs = set(conn[np.any(conn == c, axis=1)].ravel()) - {c}
        mids = [np.argmin(np.abs(mf.xyz - (mc.xyz[c] + mc.xyz[m]) / 2).sum(axis=1)) for m in nbrs]
        logs = [np.log(kf[c2f[c]])] + [0.5 * np.log(kf[f]) for f in mids]
        want = np.exp(np.sum(logs) / (1 + 0.5 * len(mids)))
        assert kc[c] == pytest.approx(want, rel=1e-13)


def test_kuhn_vertex_order_refines_as_the_path_order():
    """The Kuhn tets are listed in the vertex order (p2, p3, p0, p1) of their
    monotone path p0 -> p3; Bey's refinement in that order cuts every
    octahedron between the same midpoints as in path order, so the refined
    meshes coincide (the same set of elements, as coordinate sets, at levels
    1-3) and the faces through the cube diagonal lie opposite the first and
    last vertex."""
    for fn in (kuhn_cube, kuhn_cube_2x2x2):
        X, T = fn()
        path = T[:, [2, 3, 0, 1]]
        d = X[path[:, 1:]] - X[path[:, :-1]]
        assert np.allclose(np.abs(d).sum(axis=2), 1.0 / (2 if fn is kuhn_cube_2x2x2 else 1))
        for L in (1, 2, 3):
            sets = []
            for TT in (T, path):
                m = O.Mesh(X, TT, L)
                conn, _ = m.elements()
                P = np.rint(m.xyz[conn] * 2 ** (L + 1)).astype(np.int64)
                sets.append({tuple(sorted(map(tuple, e))) for e in P})
            assert sets[0] == sets[1], (fn.__name__, L)


def test_cube12_orientation_keeps_the_refinement():
    """cube12 lists its tets in the orders chosen by
    orient_for_contiguous_faces; each keeps the tet's vertex pairs {v0, v2},
    {v1, v3} at positions {0, 2} and {1, 3}, so the refined mesh equals that
    of the positively oriented listing (identical element sets at levels
    1-3), and 11 of the 18 shared faces lie opposite positions 0 or 3 in both
    tets (6 before)."""
    from hhg_inputs.meshes import cube12_oriented_positive
    X, T = cube12()
    X0, P = cube12_oriented_positive()
    assert np.array_equal(X, X0)
    for a, b in zip(T, P):
        pairs = lambda t: {frozenset((int(t[0]), int(t[2]))), frozenset((int(t[1]), int(t[3])))}
        assert pairs(a) == pairs(b)
    for L in (1, 2, 3):
        sets = []
        for TT in (T, P):
            m = O.Mesh(X, TT, L)
            conn, _ = m.elements()
            Q = np.rint(m.xyz[conn] * 2 ** (L + 1)).astype(np.int64)
            sets.append({tuple(sorted(map(tuple, e))) for e in Q})
        assert sets[0] == sets[1], L

    def contiguous_shared(TT):
        faces = {}
        for t in range(len(TT)):
            for q in range(4):
                faces.setdefault(tuple(sorted(np.delete(TT[t], q))), []).append(q)
        return sum(1 for v in faces.values() if len(v) == 2 and all(q in (0, 3) for q in v))
    assert contiguous_shared(T) == 11 and contiguous_shared(P) == 6
