"""The seeded input generators: their torch versions (used for node sets too
large for numpy) give the numpy versions' values, and the tensor fields
describe SPD tensors."""
import numpy as np
import pytest

from hhg_inputs import (lognormal_params, lognormal_k, lognormal_k_torch, tensor_K, tensor_fields,
                        tensor_fields_torch, polynomial_tensor_K, polynomial_tensor_fields_torch, TENSOR_DIRS,
                        kuhn_cube, kuhn_cube_2x2x2, cube12)

torch = pytest.importorskip("torch")


def _pts(n=2000, seed=0):
    return np.random.default_rng(seed).uniform(0.0, 1.0, (n, 3))


def test_torch_generators_match_numpy():
    x = _pts()
    prm = lognormal_params(3, 1.2, 0.1)
    a = lognormal_k(x, prm)
    b = lognormal_k_torch(x, lognormal_params(3, 1.2, 0.1), torch, device="cpu").numpy()
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
    a = tensor_fields(tensor_K(x))
    b = tensor_fields_torch(x, torch, device="cpu").numpy()
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
    a = tensor_fields(polynomial_tensor_K(x))
    b = polynomial_tensor_fields_torch(x, torch, device="cpu").numpy()
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()


@pytest.mark.parametrize("Kfun", [tensor_K, polynomial_tensor_K])
def test_tensor_fields_recompose_an_spd_K(Kfun):
    """sum_m k_m c_m c_m^T gives K back, and K is SPD on the unit cube."""
    x = _pts(500, 1)
    K = Kfun(x)
    k6 = tensor_fields(K)
    C = np.asarray(TENSOR_DIRS, dtype=np.float64)
    R = np.einsum("mn,mi,mj->nij", k6, C, C)
    assert np.abs(R - K).max() <= 1e-13 * np.abs(K).max()
    assert np.abs(K - np.transpose(K, (0, 2, 1))).max() <= 1e-15 * np.abs(K).max()
    assert np.linalg.eigvalsh(K).min() > 0.0


def test_2d_macro_meshes_are_conforming_and_counter_clockwise():
    from hhg_inputs import MESHES2D
    for name, fn in MESHES2D.items():
        X, T = fn()
        e1, e2 = X[T[:, 1]] - X[T[:, 0]], X[T[:, 2]] - X[T[:, 0]]
        assert np.all(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0] > 0), name
        count = {}
        for t in T:
            for a in range(3):
                e = tuple(sorted((int(t[a]), int(t[(a + 1) % 3]))))
                count[e] = count.get(e, 0) + 1
        assert max(count.values()) <= 2, name
        # the boundary edges close into the outline of the domain (Euler: V - E + F = 1)
        assert X.shape[0] - len(count) + T.shape[0] == 1, name


def _faces_contiguous_in_both(T):
    """Shared macro faces and how many of them lie on contiguous slot runs in
    both their tets.  In the slot layout (planes k, anti-diagonals s = i + j,
    index i; i, j, k the weights of the tet's vertices 1..3) the runs are the
    plane k = 0 (the face opposite the last vertex) and the last anti-diagonal
    of every plane, where vertex 0's weight is 0 (the face opposite the first
    vertex)."""
    faces = {}
    for tet in np.asarray(T):
        for q in range(4):
            faces.setdefault(tuple(sorted(np.delete(tet, q))), []).append(q)
    shared = [qs for qs in faces.values() if len(qs) == 2]
    return sum(all(q in (0, 3) for q in qs) for qs in shared), len(shared)


@pytest.mark.parametrize("mesh_fn,want", [(kuhn_cube, (6, 6)), (kuhn_cube_2x2x2, (48, 72)), (cube12, (11, 18))])
def test_shared_faces_on_contiguous_slot_runs(mesh_fn, want):
    """The listed vertex orders put the counted shared faces on contiguous runs
    in both tets; a tet has two such faces, so no listing gets more than one
    per tet (the 6- and 48-tet cubes reach that bound)."""
    X, T = mesh_fn()
    got = _faces_contiguous_in_both(T)
    assert got == want
    assert got[0] <= len(T)
