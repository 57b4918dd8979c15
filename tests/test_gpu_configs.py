"""The workload configurations at (or towards) their real shapes, through the
C ABI, checked against the CPU oracle:

* C3: 6-tet Kuhn cube, smooth k, manufactured u = sin sin sin, rhs M I_h f:
  GPU multigrid solutions to 1e-8 converge at the optimal rates (Lemma 3.1:
  O(h^2) in L2, O(h) in H1; exact errors by the oracle's quadrature).
* C4 geometry: 48 Kuhn tets, lognormal k (sigma 1.5, l_c 0.05, seed 2):
  sampled rows of both operators at level 6 (2.1M nodes, every inter-tet
  primitive kind, the 24-tet centre vertex), FP64 and FP32; FP64 and
  FP32-in-FP64 solves to 1e-10 against the oracle's sparse direct solution.
* C5: the trained weights shipped with the package on a held-out field.
"""
import numpy as np
import pytest

from hhg_inputs import (kuhn_cube, kuhn_cube_2x2x2, smooth_k, lognormal_params, lognormal_k,
                        lognormal_k_torch, uniform_vector, manufactured_u, manufactured_f, tensor_K, tensor_fields,
                        tensor_fields_torch)
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1709_06793_amd import hhg  # noqa: E402
from paper_1709_06793_amd import learned_train as LT  # noqa: E402


def _dev(x, dtype=torch.float64):
    return torch.tensor(x, dtype=dtype, device="cuda")


def _grad_u(x):
    p = np.pi
    return p * np.stack([np.cos(p * x[:, 0]) * np.sin(p * x[:, 1]) * np.sin(p * x[:, 2]),
                         np.sin(p * x[:, 0]) * np.cos(p * x[:, 1]) * np.sin(p * x[:, 2]),
                         np.sin(p * x[:, 0]) * np.sin(p * x[:, 1]) * np.cos(p * x[:, 2])], axis=1)


def _c3_solve(level):
    X, T = kuhn_cube()
    om = O.Mesh(X, T, level)
    b = O.assemble_mass(om) @ manufactured_f(om.xyz)
    b[om.dirichlet] = 0.0
    ctx = hhg.Context(X, T, level)
    ctx.set_coefficient(smooth_k(om.xyz))
    u = ctx.vector(level)
    st = ctx.solve(level, ctx.from_canonical(level, _dev(b)), u, mode=hhg.SOLVE_F64, tol=1e-8, max_iter=100)
    print(f"C3 level {level}: {st}", flush=True)
    assert st["rel_residual"] <= 1e-8 and st["status"] == 0
    return om, b, ctx.to_canonical(level, u).cpu().numpy(), st


def test_c3_rates_from_gpu_solutions():
    errs, nodal = [], []
    for level in (3, 4, 5, 6):
        om, b, uh, st = _c3_solve(level)
        e = uh - manufactured_u(om.xyz)
        h = 1.0 / 2 ** level
        nodal.append(np.sqrt(h ** 3 * np.sum(e[om.unknowns] ** 2)))
        if level <= 5:
            errs.append(O.errors(om, uh, manufactured_u, _grad_u))
        if level == 5:
            # the GPU solution solves the oracle's system: FP64 residual of the
            # oracle's own CSR operator
            op = O.make_operator(om, smooth_k(om.xyz), "scaled", modification=True)
            r = b[om.unknowns] - op.A @ uh[om.unknowns]
            assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(b[om.unknowns])
    eoc_l2 = [np.log2(a["L2"] / c["L2"]) for a, c in zip(errs, errs[1:])]
    eoc_h1 = [np.log2(a["H1"] / c["H1"]) for a, c in zip(errs, errs[1:])]
    eoc_nd = [np.log2(a / c) for a, c in zip(nodal, nodal[1:])]
    print("eoc L2", eoc_l2, "H1", eoc_h1, "nodal L2", eoc_nd, flush=True)
    assert abs(eoc_l2[-1] - 2.0) < 0.15 and abs(eoc_h1[-1] - 1.0) < 0.1
    assert abs(eoc_nd[-1] - 2.0) < 0.15


def test_c3_nodal_rates_at_levels_7_and_8():
    """C3 at its largest levels: GPU multigrid solutions (FP64, V(2,2), 1e-8)
    on the 6-tet cube with b = M I_h f (consistent mass, on the Freudenthal
    grid), nodal L2 error against u* = sin sin sin; the error falls as h^2
    (Lemma 3.1) from level 6 to 7 to 8."""
    from hhg_inputs import kuhn_cube_mass_rhs
    X, T = kuhn_cube()
    nodal = []
    for level in (6, 7, 8):
        ctx = hhg.Context(X, T, level)
        xyz, dirichlet = ctx.node_coords(level)
        ctx.set_coefficient(smooth_k(xyz))
        b = kuhn_cube_mass_rhs(xyz, level, manufactured_f)
        b[dirichlet] = 0.0
        u = ctx.vector(level)
        st = ctx.solve(level, ctx.from_canonical(level, _dev(b)), u, mode=hhg.SOLVE_F64, tol=1e-8, max_iter=100)
        print(f"C3 level {level}: {st}", flush=True)
        assert st["rel_residual"] <= 1e-8 and st["status"] == 0
        uh = ctx.to_canonical(level, u).cpu().numpy()
        e = uh - manufactured_u(xyz)
        h = 1.0 / 2 ** level
        nodal.append(np.sqrt(h ** 3 * np.sum(e[~dirichlet] ** 2)))
        ctx.close()
        del ctx, u, uh, e, b, xyz
        torch.cuda.empty_cache()
    eoc = [np.log2(a / c) for a, c in zip(nodal, nodal[1:])]
    print("nodal L2 errors", nodal, "eoc", eoc, flush=True)
    assert all(abs(x - 2.0) < 0.1 for x in eoc), eoc


def _c4_k(x):
    return lognormal_k(x, lognormal_params(2, 1.5, 0.05))


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 4e-6)])
def test_c4_geometry_sampled_rows(dtype, tol):
    X, T = kuhn_cube_2x2x2()
    level = 6
    om = O.Mesh(X, T, level)
    k = _c4_k(om.xyz)
    u = uniform_vector(om.n_nodes, seed=11)
    u[om.dirichlet] = 0.0
    ctx = hhg.Context(X, T, level)
    ctx.set_coefficient(k)
    print(f"C4 geometry level {level}: {om.n_nodes} nodes, {dtype}", flush=True)
    ud = ctx.from_canonical(level, _dev(u, dtype))
    rng = np.random.default_rng(7)
    # random rows plus every node on an inter-tet primitive near the centre
    centre = np.where(np.abs(om.xyz - 0.5).max(axis=1) <= 2.5 / 2 ** (level + 1))[0]
    nodes = np.unique(np.concatenate([rng.choice(om.n_nodes, 300, replace=False), centre]))
    uu = u.astype(np.float32).astype(np.float64) if dtype == torch.float32 else u
    for kind in ("scaled", "nodal"):
        y = ctx.vector(level, dtype)
        (ctx.apply_scaled if kind == "scaled" else ctx.apply_nodal)(level, ud, y)
        got = ctx.to_canonical(level, y).cpu().numpy().astype(np.float64)
        ref = O.apply_rows(om, k, uu, nodes, kind)
        assert np.abs(got[nodes] - ref).max() <= tol * np.abs(ref).max(), kind
        assert np.all(got[om.dirichlet] == 0.0)


def test_c4_full_size_sampled_rows():
    """48 Kuhn tets at level 8 (135M nodes, 3.3 GB FP64 working set), the
    launch the default policy makes there (the LDS-staged scaled march):
    sampled rows against the oracle's row-by-row evaluation (random rows and
    every node near the 24-tet centre vertex), the whole output against the
    two-rows-per-lane march, and zero interior rows for a constant input."""
    X, T = kuhn_cube_2x2x2()
    level = 8
    om = O.Mesh(X, T, level)
    print(f"C4 full size level {level}: {om.n_nodes} nodes", flush=True)
    k = lognormal_k_torch(om.xyz, lognormal_params(2, 1.5, 0.05), torch).cpu().numpy()
    u = uniform_vector(om.n_nodes, seed=12)
    u[om.dirichlet] = 0.0
    ctx = hhg.Context(X, T, level)
    ctx.set_coefficient(k)
    ud = ctx.from_canonical(level, _dev(u))
    rng = np.random.default_rng(8)
    centre = np.where(np.abs(om.xyz - 0.5).max(axis=1) <= 2.5 / 2 ** (level + 1))[0]
    nodes = np.unique(np.concatenate([rng.choice(om.n_nodes, 300, replace=False), centre]))
    y0, y1 = ctx.vector(level), ctx.vector(level)
    try:
        hhg.set_kernel_variant(0)
        ctx.apply_scaled(level, ud, y0)
        hhg.set_kernel_variant(6)
        ctx.apply_scaled(level, ud, y1)
    finally:
        hhg.set_kernel_variant(0)
    got = ctx.to_canonical(level, y0).cpu().numpy()
    ref = O.apply_rows(om, k, u, nodes, "scaled")
    assert np.abs(got[nodes] - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(got[om.dirichlet] == 0.0)
    d = (y1 - y0).abs().max().item() / y0.abs().max().item()
    print(f"LDS march vs two-row march: max rel difference {d:.3e}", flush=True)
    assert d <= 1e-12
    del y1, ud
    one = ctx.from_canonical(level, _dev(np.where(om.dirichlet, 0.0, 1.0)))
    ctx.apply_scaled(level, one, y0)
    v = ctx.to_canonical(level, y0).cpu().numpy()
    h = 1.5 / 2 ** (level + 1)
    inner = (om.xyz.min(axis=1) > h) & (om.xyz.max(axis=1) < 1 - h)
    assert np.abs(v[inner]).max() <= 1e-13 * np.abs(v).max()


def test_c4_tensor_full_size_sampled_rows():
    """48 Kuhn tets at level 8 with the rotating SPD tensor K (six component
    fields, 6.5 GB FP64 on the finest level), both tensor applies in the
    launches bench.py times: sampled rows (random and every node near the
    24-tet centre vertex) against the oracle's row-by-row evaluation, zero
    Dirichlet rows, and the FP32 applies against the FP64 ones."""
    X, T = kuhn_cube_2x2x2()
    level = 8
    om = O.Mesh(X, T, level)
    print(f"C4 tensor full size level {level}: {om.n_nodes} nodes", flush=True)
    u = uniform_vector(om.n_nodes, seed=13)
    u[om.dirichlet] = 0.0
    ctx = hhg.Context(X, T, level)
    ctx.set_tensor_coefficient(tensor_fields_torch(om.xyz, torch))
    ud = ctx.from_canonical(level, _dev(u))
    rng = np.random.default_rng(9)
    centre = np.where(np.abs(om.xyz - 0.5).max(axis=1) <= 2.5 / 2 ** (level + 1))[0]
    nodes = np.unique(np.concatenate([rng.choice(om.n_nodes, 200, replace=False), centre]))
    y = ctx.vector(level)
    for form, apply in (("scaled", ctx.apply_tensor), ("nodal", ctx.apply_tensor_nodal)):
        apply(level, ud, y)
        got = ctx.to_canonical(level, y).cpu().numpy()
        ref = O.apply_tensor_rows(om, lambda x: tensor_fields(tensor_K(x)), u, nodes, form)
        err = np.abs(got[nodes] - ref).max() / np.abs(ref).max()
        print(f"tensor {form}: {len(nodes)} sampled rows, max rel error {err:.3e}", flush=True)
        assert err <= 1e-12, form
        assert np.all(got[om.dirichlet] == 0.0), form
        # FP32 at the same size: within FP32 rounding of the FP64 result
        y32 = ctx.vector(level, torch.float32)
        apply(level, ud.float(), y32)
        d = ((y32.double() - y).abs().max() / y.abs().max()).item()
        print(f"tensor {form} FP32 vs FP64: max rel difference {d:.3e}", flush=True)
        assert d <= 4e-6, form
        del y32


@pytest.mark.parametrize("mode", [hhg.SOLVE_F64, hhg.SOLVE_MIXED])
def test_c4_solve_to_1e10_matches_oracle(mode):
    import scipy.sparse.linalg as spla
    X, T = kuhn_cube_2x2x2()
    level = 4
    om = O.Mesh(X, T, level)
    k = _c4_k(om.xyz)
    f = uniform_vector(om.n_nodes, seed=2)
    f[om.dirichlet] = 0.0
    ctx = hhg.Context(X, T, level)
    ctx.set_coefficient(k)
    u = ctx.vector(level)
    st = ctx.solve(level, ctx.from_canonical(level, _dev(f)), u, mode=mode, tol=1e-10, max_iter=80)
    print(f"C4 level {level} mode {mode}: {st}", flush=True)
    assert st["rel_residual"] <= 1e-10 and st["status"] == 0
    op = O.make_operator(om, k, "scaled", modification=True)
    ref = np.zeros(om.n_nodes)
    ref[om.unknowns] = spla.spsolve(op.A.tocsc(), f[om.unknowns])
    got = ctx.to_canonical(level, u).cpu().numpy()
    r = f[om.unknowns] - op.A @ got[om.unknowns]
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(f[om.unknowns])
    assert np.linalg.norm(got - ref) <= 1e-7 * np.linalg.norm(ref)


def test_c5_shipped_weights_on_held_out_field():
    w, meta = LT.load_weights()
    assert meta["fields"] == [100, 355] and meta["level"] == 6
    ctx, f, prm = LT.make_field_context(5, 1005, kuhn_cube, torch)
    res = LT.evaluate(ctx, f, 5, w, torch)
    print("C5 held-out field 1005 at level 5:", res, flush=True)
    # with the default fallback (learned cycles must contract within 1.05 x
    # the plain cycle measured from the same iterate) the solve converges and
    # is never much worse than plain Chebyshev
    assert res["learned"]["rel_residual"] <= 1e-8
    assert res["learned"]["iterations"] <= res["chebyshev"]["iterations"] + 1
    # the network alone (no comparison with the plain cycle): converges
    # without falling back and beats the same cycles with the network off
    ctx.learned_set_weights(w)
    ctx.learned_set_fallback(1.0, 0.0)
    u = ctx.vector(5)
    st = ctx.solve(5, f, u, mode=hhg.SOLVE_LEARNED, tol=1e-8, max_iter=200)
    print("network alone:", st, flush=True)
    assert st["fallback"] == 0 and st["rel_residual"] <= 1e-8
    assert st["iterations"] < res["network_off"]["iterations"]
