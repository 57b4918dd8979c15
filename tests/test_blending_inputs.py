"""Pins of the blending example's inputs (Sec. 7.4, the half cylinder mantle
on its reference box), CPU only: the mapping tensor against the Jacobian of
the mapping Phi taken by finite differences, the right-hand side against a
finite-difference divergence of the flux, the boundary values of the
manufactured solution, and the grid mass right-hand side against the oracle's
assembled mass matrix."""
import numpy as np

from hhg_inputs import (CYLINDER_BOX, cylinder_reference_box, kuhn_box, kuhn_box_mass_rhs, cylinder_mapping_K,
                        cylinder_phi, cylinder_phi_inverse, cylinder_tensor, cylinder_u, cylinder_f,
                        tensor_fields)
from oracle import oracle as O


def _box_points(n, seed, margin=0.01):
    lo, hi = (np.asarray(a, dtype=np.float64) for a in CYLINDER_BOX)
    rng = np.random.default_rng(seed)
    return lo + (hi - lo) * rng.uniform(margin, 1 - margin, (n, 3))


def _d(fun, x, axis, h):
    """Fourth-order central difference of fun along `axis` at the points x."""
    e = np.zeros(3)
    e[axis] = h
    return (-fun(x + 2 * e) + 8 * fun(x + e) - 8 * fun(x - e) + fun(x - 2 * e)) / (12 * h)


def test_mapping_tensor_is_the_jacobian_expression():
    """K = (D Phi)(D Phi)^T / |det D Phi| at x = Phi^{-1}(xh), with D Phi taken
    by central differences of Phi (the mapping itself, not the closed form of
    K), and Phi(Phi^{-1}(xh)) = xh."""
    xh = _box_points(200, 1)
    xp = cylinder_phi_inverse(xh)
    assert np.abs(cylinder_phi(xp) - xh).max() < 1e-13
    J = np.stack([_d(cylinder_phi, xp, a, 1e-4) for a in range(3)], axis=2)   # J[:, i, a] = d Phi_i / d x_a
    Kn = J @ np.transpose(J, (0, 2, 1)) / np.abs(np.linalg.det(J))[:, None, None]
    K = cylinder_mapping_K(xh)
    assert np.abs(K - Kn).max() < 1e-9 * np.abs(K).max()
    assert np.all(np.linalg.eigvalsh(K) > 0)
    assert np.allclose(cylinder_tensor(xh), (1 + xh[:, 2])[:, None, None] * K, rtol=1e-15, atol=0)


def test_rhs_is_minus_divergence_of_the_flux():
    """f = -div((1 + z) K grad u) against nested finite differences: grad u of
    cylinder_u numerically, the flux with the tensor, its divergence
    numerically."""
    xh = _box_points(100, 2, margin=0.05)
    h = 2e-3

    def flux(x, i):
        g = np.stack([_d(cylinder_u, x, a, h) for a in range(3)], axis=1)
        return np.einsum("nj,nj->n", cylinder_tensor(x)[:, i, :], g)

    div = sum(_d(lambda x, i=i: flux(x, i), xh, i, h) for i in range(3))
    f = cylinder_f(xh)
    assert np.abs(f + div).max() < 1e-6 * np.abs(f).max()


def test_manufactured_solution_vanishes_on_the_box_boundary():
    lo, hi = (np.asarray(a, dtype=np.float64) for a in CYLINDER_BOX)
    x = _box_points(300, 3, margin=0.0)
    for d in range(3):
        for v in (lo[d], hi[d]):
            y = x.copy()
            y[:, d] = v
            assert np.abs(cylinder_u(y)).max() < 1e-14
    assert np.abs(cylinder_u(_box_points(300, 4))).max() > 0.5


def test_kuhn_box_is_conforming_and_its_mass_rhs_matches_the_oracle():
    """The Kuhn box's refinement is the Freudenthal triangulation of the fine
    grid (every fine node on the grid), and the grid-stencil b = M I_h f
    equals the oracle's assembled mass matrix times f on every unknown."""
    X, T = cylinder_reference_box((1, 2, 3))
    lo, hi = CYLINDER_BOX
    for L in (1, 2):
        m = O.Mesh(X, T, L)
        N = np.array((1, 2, 3)) * 2 ** L
        g = (m.xyz - np.asarray(lo)) / ((np.asarray(hi) - np.asarray(lo)) / N)
        assert np.abs(g - np.rint(g)).max() < 1e-9
        assert m.n_nodes == np.prod(N + 1)
        want = O.assemble_mass(m) @ cylinder_f(m.xyz)
        got = kuhn_box_mass_rhs(m.xyz, L, cylinder_f, (1, 2, 3), lo, hi)
        u = m.unknowns
        assert np.abs(got[u] - want[u]).max() <= 1e-13 * np.abs(want[u]).max()
    Xb, Tb = kuhn_box((2, 1, 1), (0, 0, 0), (2.0, 1.0, 1.0))
    assert len(Tb) == 12 and Xb.shape == (12, 3)


def test_blending_tensor_discretisation_converges_at_second_order():
    """The oracle's scaled tensor operator with (1 + z) K on the reference box,
    solved directly against b = M I_h f: the nodal L2 error against u*
    decreases at second order (Sec. 7.4 reports eoc 2)."""
    import scipy.sparse.linalg as spla
    X, T = cylinder_reference_box((1, 2, 2))
    lo, hi = CYLINDER_BOX
    errs = []
    for L in (3, 4):
        m = O.Mesh(X, T, L)
        op = O.make_tensor_operator(m, tensor_fields(cylinder_tensor(m.xyz)), "scaled")
        b = kuhn_box_mass_rhs(m.xyz, L, cylinder_f, (1, 2, 2), lo, hi)
        u = np.zeros(m.n_nodes)
        u[m.unknowns] = spla.spsolve(op.A.tocsc(), b[m.unknowns])
        vol = np.prod((np.asarray(hi) - np.asarray(lo)) / (np.array((1, 2, 2)) * 2 ** L))
        errs.append(np.sqrt(vol * np.sum((u - cylinder_u(m.xyz)) ** 2)))
    eoc = np.log2(errs[0] / errs[1])
    assert 1.7 < eoc < 2.5, (errs, eoc)
