"""Parity of the HIP path (through the C ABI) with the CPU oracle.

FP64 tolerance: 1e-12 relative, norm-wise and element-wise against the
largest entry (the target the method's precision statement fixes).  FP32:
bounded by the FP32 rounding of inputs and of 15-term sums (a few 1e-6 relative).
"""
import numpy as np
import pytest

from hhg_inputs import (unit_tet, regular_tet, flat_tet, kuhn_cube, kuhn_cube_2x2x2, cube12, smooth_k,
                        sigmoid_k, lognormal_params, lognormal_k, uniform_vector, affine_k, tensor_K,
                        tensor_fields, polynomial_tensor_K)
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1709_06793_amd import hhg  # noqa: E402

TOL64 = 1e-12


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _elem(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _setup(mesh_fn, level, kfun=smooth_k, seed=0, flags=0):
    X, T = mesh_fn()
    om = O.Mesh(X, T, level)
    k = kfun(om.xyz)
    u = uniform_vector(om.n_nodes, seed=seed)
    u[om.dirichlet] = 0.0
    ctx = hhg.Context(X, T, level, flags)
    ctx.set_coefficient(k)
    print(f"case {mesh_fn.__name__} level {level}", flush=True)
    return om, k, u, ctx


def _dev(x, dtype=torch.float64):
    return torch.tensor(x, dtype=dtype, device="cuda")


CASES = [(unit_tet, 4), (unit_tet, 5), (regular_tet, 4), (kuhn_cube, 3), (kuhn_cube, 4),
         (kuhn_cube_2x2x2, 2), (kuhn_cube_2x2x2, 3), (flat_tet, 4)]


@pytest.mark.parametrize("mesh_fn,level", CASES)
@pytest.mark.parametrize("kind", ["scaled", "nodal"])
def test_apply_fp64_matches_oracle(mesh_fn, level, kind):
    om, k, u, ctx = _setup(mesh_fn, level, flags=hhg.FLAG_NO_MODIFICATION)
    y = ctx.vector(level)
    ud = ctx.from_canonical(level, _dev(u))
    (ctx.apply_scaled if kind == "scaled" else ctx.apply_nodal)(level, ud, y)
    got = ctx.to_canonical(level, y).cpu().numpy()
    ref = O.make_operator(om, k, kind).apply(u)
    assert _rel(got, ref) <= TOL64 and _elem(got, ref) <= TOL64, (_rel(got, ref), _elem(got, ref))
    assert np.all(got[om.dirichlet] == 0.0)


@pytest.mark.parametrize("mesh_fn,level", [(unit_tet, 5), (kuhn_cube_2x2x2, 3), (flat_tet, 4), (kuhn_cube, 6)])
@pytest.mark.parametrize("variant", [1, 6, 10])
def test_apply_fp64_kernel_variants(mesh_fn, level, variant):
    """Every interior-kernel variant the default policy can choose (1: one row
    per lane, 6: two rows per lane, 10: LDS-staged blocks), forced, with the
    modification on: the oracle's operator, and the default variant's output."""
    om, k, u, ctx = _setup(mesh_fn, level, kfun=lambda x: lognormal_k(x, lognormal_params(3, 1.5, 0.1)))
    ud = ctx.from_canonical(level, _dev(u))
    y0, y1 = ctx.vector(level), ctx.vector(level)
    try:
        hhg.set_kernel_variant(0)
        ctx.apply_scaled(level, ud, y0)
        hhg.set_kernel_variant(variant)
        ctx.apply_scaled(level, ud, y1)
    finally:
        hhg.set_kernel_variant(0)
    got = ctx.to_canonical(level, y1).cpu().numpy()
    ref = O.make_operator(om, k, "scaled", modification=True).apply(u)
    assert _rel(got, ref) <= TOL64 and _elem(got, ref) <= TOL64, (_rel(got, ref), _elem(got, ref))
    assert np.all(got[om.dirichlet] == 0.0)
    d = (y1 - y0).abs().max().item() / y0.abs().max().item()
    print(f"variant {variant} vs default: max rel difference {d:.3e}", flush=True)
    assert d <= TOL64


@pytest.mark.parametrize("mesh_fn,level", [(unit_tet, 5), (kuhn_cube_2x2x2, 3), (flat_tet, 4), (kuhn_cube, 6)])
@pytest.mark.parametrize("variant", [1, 6, 10])
def test_apply_fp32_kernel_variants(mesh_fn, level, variant):
    """The FP32 interior-kernel variants (1: one row per lane, 6: two rows
    per lane, 10: LDS-staged blocks), forced, with the modification on: the
    oracle's operator on the FP32-rounded u and k (2e-6), and the default
    variant's output."""
    om, k, u, ctx = _setup(mesh_fn, level, kfun=lambda x: lognormal_k(x, lognormal_params(3, 1.5, 0.1)))
    u32 = u.astype(np.float32).astype(np.float64)
    k32 = k.astype(np.float32).astype(np.float64)
    ud = ctx.from_canonical(level, _dev(u32).float())
    y0, y1 = ctx.vector(level, torch.float32), ctx.vector(level, torch.float32)
    try:
        hhg.set_kernel_variant(0)
        ctx.apply_scaled(level, ud, y0)
        hhg.set_kernel_variant(variant)
        ctx.apply_scaled(level, ud, y1)
    finally:
        hhg.set_kernel_variant(0)
    got = ctx.to_canonical(level, y1).cpu().numpy().astype(np.float64)
    mods, _ = O.modification_factors(om, k)
    ref = O.Operator(om, O.assemble(om, k32, "scaled", mods=mods)).apply(u32)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"FP32 variant {variant}: max error {err:.2e} of the largest row", flush=True)
    assert err <= 2e-6
    assert np.all(got[om.dirichlet] == 0.0)
    d = (y1 - y0).abs().max().item() / y0.abs().max().item()
    assert d <= 2e-6


@pytest.mark.parametrize("mesh_fn,level", [(unit_tet, 5), (kuhn_cube_2x2x2, 3), (flat_tet, 4), (kuhn_cube, 6)])
def test_fp32_lds_residual_and_chebyshev(mesh_fn, level):
    """The LDS-staged block march in the FP32 residual (with its block norms)
    and the fused Chebyshev sweep, forced (variant 10), with the modification
    on: the residual against the oracle's on the FP32-rounded u, f and k
    (2e-6 of the largest of |f| and |Au|) and its norm against the default
    kernel's; three sweeps against the default kernel's (1e-5) and a
    FP32-in-FP64 solve to 1e-10 against the default kernel's solution."""
    om, k, u, ctx = _setup(mesh_fn, level, kfun=lambda x: lognormal_k(x, lognormal_params(3, 1.5, 0.1)))
    f = uniform_vector(om.n_nodes, seed=17)
    f[om.dirichlet] = 0.0
    u32, f32, k32 = (a.astype(np.float32).astype(np.float64) for a in (u, f, k))
    mods, _ = O.modification_factors(om, k)
    op32 = O.Operator(om, O.assemble(om, k32, "scaled", mods=mods))
    Au = op32.apply(u32)
    ref = f32 - Au
    ref[om.dirichlet] = 0.0
    ud, fd = ctx.from_canonical(level, _dev(u32).float()), ctx.from_canonical(level, _dev(f32).float())
    out = {}
    try:
        for v in (0, 10):
            hhg.set_kernel_variant(v)
            r = ctx.vector(level, torch.float32)
            nrm = ctx.residual(level, fd, ud, r, norm=True)
            w = ud.clone()
            ctx.smooth(level, fd, w, 3, hhg.CHEBYSHEV)
            x = ctx.vector(level)
            st = ctx.solve(level, ctx.from_canonical(level, _dev(f)), x, mode=hhg.SOLVE_MIXED, tol=1e-10,
                           max_iter=80)
            out[v] = (ctx.to_canonical(level, r).cpu().numpy().astype(np.float64), nrm,
                      ctx.to_canonical(level, w).cpu().numpy().astype(np.float64), st,
                      ctx.to_canonical(level, x).cpu().numpy())
    finally:
        hhg.set_kernel_variant(0)
    r10, n10, w10, st10, x10 = out[10]
    r0, n0, w0, st0, x0 = out[0]
    scale = max(np.abs(f32).max(), np.abs(Au).max())
    err = np.abs(r10 - ref).max() / scale
    print(f"FP32 LDS residual: max error {err:.2e}; norms {n10:.6e} {n0:.6e}", flush=True)
    assert err <= 2e-6
    assert np.all(r10[om.dirichlet] == 0.0)
    assert n10 == pytest.approx(n0, rel=1e-5)
    assert np.linalg.norm(w10 - w0) <= 1e-5 * np.linalg.norm(w0)
    assert st10["status"] == 0 and st10["rel_residual"] <= 1e-10
    assert np.linalg.norm(x10 - x0) <= 1e-8 * np.linalg.norm(x0)


MIX = [(3, (0, 1)), (7, (0, 1, 2)), (4, (2,)), (1, (0,)), (0, ())]


@pytest.mark.parametrize("mesh_fn,level", [(cube12, 3), (cube12, 4), (kuhn_cube_2x2x2, 3), (unit_tet, 4)])
@pytest.mark.parametrize("mask,dims", MIX)
def test_apply_mixed_fp64_matches_oracle(mesh_fn, level, mask, dims):
    """Sec. 5 eq. (modst): nodal-integration rows on the selected macro
    primitives, scaled rows (modification on) elsewhere."""
    om, k, u, ctx = _setup(mesh_fn, level, kfun=lambda x: lognormal_k(x, lognormal_params(4, 1.0, 0.2)))
    y = ctx.vector(level)
    ctx.apply_mixed(level, ctx.from_canonical(level, _dev(u)), y, mask)
    got = ctx.to_canonical(level, y).cpu().numpy()
    ref = O.make_mixed_operator(om, k, dims, modification=True).apply(u)
    assert _rel(got, ref) <= TOL64 and _elem(got, ref) <= TOL64, (_rel(got, ref), _elem(got, ref))
    assert np.all(got[om.dirichlet] == 0.0)


@pytest.mark.parametrize("mask,dims", [(3, (0, 1)), (7, (0, 1, 2)), (0, ())])
def test_apply_mixed_with_modification_triggered(mask, dims):
    """Steep sigmoid k on the 12-tet cube: modified edges touch vertex, edge,
    face and interior rows; rows switched to nodal integration carry no
    modification."""
    om, k, u, ctx = _setup(cube12, 3, kfun=lambda x: sigmoid_k(x, 100.0))
    assert ctx.level_info(3)["n_modified"] > 0
    y = ctx.vector(3)
    ctx.apply_mixed(3, ctx.from_canonical(3, _dev(u)), y, mask)
    got = ctx.to_canonical(3, y).cpu().numpy()
    ref = O.make_mixed_operator(om, k, dims, modification=True).apply(u)
    assert _rel(got, ref) <= TOL64 and _elem(got, ref) <= TOL64, (_rel(got, ref), _elem(got, ref))
    if mask == 0:
        # no nodal rows: the scaled operator (its shared rows run on their own
        # pattern, so the sums are ordered differently: rounding only)
        ys = ctx.vector(3)
        ctx.apply_scaled(3, ctx.from_canonical(3, _dev(u)), ys)
        assert (ys - y).abs().max().item() <= TOL64 * y.abs().max().item()


def test_apply_mixed_fp32_and_bad_mask():
    om, k, u, ctx = _setup(cube12, 4, kfun=lambda x: lognormal_k(x, lognormal_params(4, 1.0, 0.2)))
    y = ctx.vector(4, torch.float32)
    ctx.apply_mixed(4, ctx.from_canonical(4, _dev(u, torch.float32)), y, 3)
    got = ctx.to_canonical(4, y).cpu().numpy().astype(np.float64)
    ref = O.make_mixed_operator(om, k, (0, 1), modification=True).apply(u)
    assert _rel(got, ref) <= 2e-6, _rel(got, ref)
    with pytest.raises(hhg.HHGError):
        ctx.apply_mixed(4, ctx.from_canonical(4, _dev(u)), ctx.vector(4), 8)


@pytest.mark.parametrize("mesh_fn,level,kfun", [(unit_tet, 5, None), (kuhn_cube, 4, None), (kuhn_cube_2x2x2, 3, None),
                                               (cube12, 3, None), (cube12, 3, "sigmoid"), (flat_tet, 4, "sigmoid")])
def test_apply_stored_matches_oracle(mesh_fn, level, kfun):
    """Stored stencils (15 coefficients per interior row) against the
    oracle's scaled operator, FP64 and FP32, modification included; refreshed
    by a new coefficient."""
    kf = (lambda x: sigmoid_k(x, 100.0)) if kfun == "sigmoid" else (lambda x: lognormal_k(x, lognormal_params(5, 1.0, 0.2)))
    om, k, u, ctx = _setup(mesh_fn, level, kfun=kf)
    if kfun == "sigmoid":
        assert ctx.level_info(level)["n_modified"] > 0
    with pytest.raises(hhg.HHGError):
        ctx.apply_stored(level, ctx.from_canonical(level, _dev(u)), ctx.vector(level))
    ctx.store_stencils(level)
    ref = O.make_operator(om, k, "scaled", modification=True).apply(u)
    y = ctx.vector(level)
    ctx.apply_stored(level, ctx.from_canonical(level, _dev(u)), y)
    got = ctx.to_canonical(level, y).cpu().numpy()
    assert _rel(got, ref) <= TOL64 and _elem(got, ref) <= TOL64, (_rel(got, ref), _elem(got, ref))
    assert np.all(got[om.dirichlet] == 0.0)
    y32 = ctx.vector(level, torch.float32)
    ctx.apply_stored(level, ctx.from_canonical(level, _dev(u, torch.float32)), y32)
    got32 = ctx.to_canonical(level, y32).cpu().numpy().astype(np.float64)
    assert _rel(got32, ref) <= 2e-6, _rel(got32, ref)
    k2 = smooth_k(om.xyz)
    ctx.set_coefficient(k2)
    ctx.apply_stored(level, ctx.from_canonical(level, _dev(u)), y)
    got = ctx.to_canonical(level, y).cpu().numpy()
    ref = O.make_operator(om, k2, "scaled", modification=True).apply(u)
    assert _rel(got, ref) <= TOL64, _rel(got, ref)


def _tensor_apply(ctx, form):
    return ctx.apply_tensor if form == "scaled" else ctx.apply_tensor_nodal


@pytest.mark.parametrize("form", ["scaled", "nodal"])
@pytest.mark.parametrize("mesh_fn,level", [(unit_tet, 4), (unit_tet, 5), (kuhn_cube, 3), (cube12, 3),
                                           (kuhn_cube_2x2x2, 3), (flat_tet, 4)])
def test_apply_tensor_matches_oracle(mesh_fn, level, form):
    """Sec. 2.1 eq. (integral), six components each scaled (or each nodally
    integrated), on a rotating SPD K field: FP64 at the finest and the next
    coarser level (fields injected), FP32.  Unit tet level 5 has two plane
    chunks, the second ragged."""
    X, T = mesh_fn()
    ctx = hhg.Context(X, T, level)
    apply = _tensor_apply(ctx, form)
    with pytest.raises(hhg.HHGError):
        apply(level, ctx.vector(level), ctx.vector(level))
    om = O.Mesh(X, T, level)
    ctx.set_tensor_coefficient(tensor_fields(tensor_K(om.xyz)))
    for lv in (level, level - 1):
        m = O.Mesh(X, T, lv)
        K6 = tensor_fields(tensor_K(m.xyz))
        u = uniform_vector(m.n_nodes, seed=3)
        u[m.dirichlet] = 0.0
        y = ctx.vector(lv)
        apply(lv, ctx.from_canonical(lv, _dev(u)), y)
        got = ctx.to_canonical(lv, y).cpu().numpy()
        ref = O.make_tensor_operator(m, K6, form).apply(u)
        assert _rel(got, ref) <= TOL64 and _elem(got, ref) <= TOL64, (lv, _rel(got, ref), _elem(got, ref))
        assert np.all(got[m.dirichlet] == 0.0)
    y32 = ctx.vector(level, torch.float32)
    u = uniform_vector(om.n_nodes, seed=3)
    u[om.dirichlet] = 0.0
    apply(level, ctx.from_canonical(level, _dev(u, torch.float32)), y32)
    got = ctx.to_canonical(level, y32).cpu().numpy().astype(np.float64)
    ref = O.make_tensor_operator(om, tensor_fields(tensor_K(om.xyz)), form).apply(u)
    assert _rel(got, ref) <= 4e-6, _rel(got, ref)


def test_apply_tensor_with_scalar_K_is_the_scalar_operator():
    """K = k I reduces the tensor operator to -div(k grad u): the scaled form
    to apply_scaled, the nodal form to apply_nodal."""
    X, T = cube12()
    level = 4
    om, k, u, ctx = _setup(cube12, level, kfun=lambda x: lognormal_k(x, lognormal_params(6, 1.0, 0.2)),
                           flags=hhg.FLAG_NO_MODIFICATION)
    ctx.set_tensor_coefficient(tensor_fields(k[:, None, None] * np.eye(3)[None]))
    ud = ctx.from_canonical(level, _dev(u))
    y1, y2 = ctx.vector(level), ctx.vector(level)
    ctx.apply_tensor(level, ud, y1)
    ctx.apply_scaled(level, ud, y2)
    assert ((y1 - y2).abs().max() / y2.abs().max()).item() <= 1e-13
    ctx.apply_tensor_nodal(level, ud, y1)
    ctx.apply_nodal(level, ud, y2)
    assert ((y1 - y2).abs().max() / y2.abs().max()).item() <= 1e-13


@pytest.mark.parametrize("mode", [hhg.SOLVE_F64, hhg.SOLVE_MIXED])
@pytest.mark.parametrize("form", ["scaled", "nodal"])
def test_solve_tensor_matches_oracle(form, mode):
    """Multigrid on the tensor operator (Sec. 7's tensor comparison) with
    either form on every level: converges to 1e-10 at a multigrid rate, and
    the result solves the oracle's matrix and matches its direct solution."""
    import scipy.sparse.linalg as spla
    X, T = cube12()
    level = 5
    om = O.Mesh(X, T, level)
    K6 = tensor_fields(tensor_K(om.xyz))
    f = uniform_vector(om.n_nodes, seed=4)
    f[om.dirichlet] = 0.0
    ctx = hhg.Context(X, T, level)
    fd, u = ctx.from_canonical(level, _dev(f)), ctx.vector(level)
    with pytest.raises(hhg.HHGError):
        ctx.solve_tensor(level, fd, u, form=form, mode=mode)
    ctx.set_tensor_coefficient(K6)
    with pytest.raises(hhg.HHGError):
        ctx.solve_tensor(level, fd, u, form=form, mode=hhg.SOLVE_LEARNED)
    st = ctx.solve_tensor(level, fd, u, form=form, mode=mode, tol=1e-10, max_iter=60, pre=3, post=3)
    print(f"tensor solve {form} mode {mode}: {st}", flush=True)
    assert st["rel_residual"] <= 1e-10 and st["status"] == 0 and st["rho"] < 0.5
    op = O.make_tensor_operator(om, K6, form)
    ref = np.zeros(om.n_nodes)
    ref[om.unknowns] = spla.spsolve(op.A.tocsc(), f[om.unknowns])
    got = ctx.to_canonical(level, u).cpu().numpy()
    r = f[om.unknowns] - op.A @ got[om.unknowns]
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(f[om.unknowns])
    assert np.linalg.norm(got - ref) <= 1e-7 * np.linalg.norm(ref)
    assert np.all(got[om.dirichlet] == 0.0)


@pytest.mark.parametrize("form", ["scaled", "nodal"])
def test_solve_tensor_polynomial_K_matches_oracle(form):
    """The polynomial permeability of the paper's tensor comparison (negative
    off-diagonal entries, so three of the six component fields are negative):
    FP64 solve to 1e-10 against the oracle's direct solution."""
    import scipy.sparse.linalg as spla
    X, T = cube12()
    level = 5
    om = O.Mesh(X, T, level)
    K6 = tensor_fields(polynomial_tensor_K(om.xyz))
    assert K6[3:].max() <= 0.0
    f = uniform_vector(om.n_nodes, seed=7)
    f[om.dirichlet] = 0.0
    ctx = hhg.Context(X, T, level)
    ctx.set_tensor_coefficient(K6)
    u = ctx.vector(level)
    st = ctx.solve_tensor(level, ctx.from_canonical(level, _dev(f)), u, form=form, tol=1e-10, max_iter=60,
                          pre=3, post=3)
    print(f"polynomial K tensor solve {form}: {st}", flush=True)
    assert st["rel_residual"] <= 1e-10 and st["status"] == 0
    op = O.make_tensor_operator(om, K6, form)
    ref = np.zeros(om.n_nodes)
    ref[om.unknowns] = spla.spsolve(op.A.tocsc(), f[om.unknowns])
    got = ctx.to_canonical(level, u).cpu().numpy()
    assert np.linalg.norm(got - ref) <= 1e-7 * np.linalg.norm(ref)


@pytest.mark.parametrize("form,mode", [("nodal", hhg.SOLVE_F64), ("nodal", hhg.SOLVE_MIXED),
                                       ("mixed", hhg.SOLVE_F64), ("mixed", hhg.SOLVE_MIXED)])
def test_solve_form_matches_oracle(form, mode):
    """Multigrid on the nodal-integration operator and on the primitive-mixed
    a_{h;I} with nodal rows on macro vertices and edges ("scale Vol+Face")
    on every level: converges to 1e-10 and matches the oracle's direct
    solution of that operator."""
    import scipy.sparse.linalg as spla
    X, T = cube12()
    level = 5
    om, k, _, ctx = _setup(cube12, level, kfun=smooth_k)
    f = uniform_vector(om.n_nodes, seed=8)
    f[om.dirichlet] = 0.0
    fd, u = ctx.from_canonical(level, _dev(f)), ctx.vector(level)
    mask = hhg.PRIM_VERTICES | hhg.PRIM_EDGES
    with pytest.raises(hhg.HHGError):
        ctx.solve_form(level, fd, u, form=form, nodal_primitives=mask, mode=hhg.SOLVE_LEARNED)
    st = ctx.solve_form(level, fd, u, form=form, nodal_primitives=mask, mode=mode, tol=1e-10, max_iter=60,
                        pre=3, post=3)
    print(f"{form} solve mode {mode}: {st}", flush=True)
    assert st["rel_residual"] <= 1e-10 and st["status"] == 0 and st["rho"] < 0.5
    op = (O.make_operator(om, k, "nodal") if form == "nodal"
          else O.make_mixed_operator(om, k, (0, 1), modification=True))
    ref = np.zeros(om.n_nodes)
    ref[om.unknowns] = spla.spsolve(op.A.tocsc(), f[om.unknowns])
    got = ctx.to_canonical(level, u).cpu().numpy()
    r = f[om.unknowns] - op.A @ got[om.unknowns]
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(f[om.unknowns])
    assert np.linalg.norm(got - ref) <= 1e-7 * np.linalg.norm(ref)
    # the scaled form through the same entry point is hhg_solve
    u2, u3 = ctx.vector(level), ctx.vector(level)
    s2 = ctx.solve_form(level, fd, u2, form="scaled", tol=1e-9, max_iter=40)
    s3 = ctx.solve(level, fd, u3, tol=1e-9, max_iter=40)
    assert s2["iterations"] == s3["iterations"] and torch.equal(u2, u3)


def test_solve_tensor_with_scalar_K_is_the_scalar_solve():
    """K = k I: the scaled tensor solve takes the scalar solve's cycles (same
    operator on every level, same diagonals and bounds up to rounding)."""
    X, T = cube12()
    level = 5
    om, k, u, ctx = _setup(cube12, level, kfun=smooth_k, flags=hhg.FLAG_NO_MODIFICATION)
    ctx.set_tensor_coefficient(tensor_fields(k[:, None, None] * np.eye(3)[None]))
    f = uniform_vector(om.n_nodes, seed=6)
    f[om.dirichlet] = 0.0
    fd = ctx.from_canonical(level, _dev(f))
    u1, u2 = ctx.vector(level), ctx.vector(level)
    s1 = ctx.solve(level, fd, u1, tol=1e-10, max_iter=60, pre=3, post=3)
    s2 = ctx.solve_tensor(level, fd, u2, tol=1e-10, max_iter=60, pre=3, post=3)
    assert s1["iterations"] == s2["iterations"] and abs(s1["rho"] - s2["rho"]) <= 1e-6, (s1, s2)
    assert ((u1 - u2).abs().max() / u1.abs().max()).item() <= 1e-9


@pytest.mark.parametrize("mesh_fn,level", [(unit_tet, 5), (kuhn_cube_2x2x2, 3)])
@pytest.mark.parametrize("kind", ["scaled", "nodal"])
def test_apply_fp32_matches_oracle(mesh_fn, level, kind):
    om, k, u, ctx = _setup(mesh_fn, level, kfun=lambda x: lognormal_k(x, lognormal_params(1, 1.0, 0.1)),
                           flags=hhg.FLAG_NO_MODIFICATION)
    y = ctx.vector(level, torch.float32)
    ud = ctx.from_canonical(level, _dev(u, torch.float32))
    (ctx.apply_scaled if kind == "scaled" else ctx.apply_nodal)(level, ud, y)
    got = ctx.to_canonical(level, y).cpu().numpy().astype(np.float64)
    ref = O.make_operator(om, k, kind).apply(u)
    assert _rel(got, ref) <= 2e-6, _rel(got, ref)


def test_c1_jacobi_sweeps_every_iterate():
    """Unit tet level 4, smooth k, u ~ U[-1,1] (seed 0), f = 0: 10 weighted
    Jacobi sweeps (omega = 2/3), each iterate against the oracle."""
    om, k, u, ctx = _setup(unit_tet, 4)
    op = O.make_operator(om, k, "scaled", modification=True)
    f = np.zeros(om.n_nodes)
    _, its = O.jacobi(op, f, u, 10, 2.0 / 3.0, history=True)
    ud = ctx.from_canonical(4, _dev(u))
    fd = ctx.vector(4)
    for s in range(10):
        ctx.smooth(4, fd, ud, 1, hhg.JACOBI, 2.0 / 3.0)
        got = ctx.to_canonical(4, ud).cpu().numpy()
        assert _rel(got, its[s]) <= TOL64, (s, _rel(got, its[s]))
    # a second right-hand side drawn after u from the same stream
    rng = np.random.default_rng(0)
    rng.uniform(-1, 1, om.n_nodes)
    f2 = rng.uniform(-1, 1, om.n_nodes)
    f2[om.dirichlet] = 0.0
    ref2 = O.jacobi(op, f2, u, 10, 2.0 / 3.0)
    ud = ctx.from_canonical(4, _dev(u))
    ctx.smooth(4, ctx.from_canonical(4, _dev(f2)), ud, 10, hhg.JACOBI, 2.0 / 3.0)
    assert _rel(ctx.to_canonical(4, ud).cpu().numpy(), ref2) <= TOL64


@pytest.mark.parametrize("mesh_fn,level", [(unit_tet, 5), (kuhn_cube_2x2x2, 3), (flat_tet, 4)])
def test_residual_and_norm(mesh_fn, level):
    om, k, u, ctx = _setup(mesh_fn, level)
    f = uniform_vector(om.n_nodes, seed=7)
    f[om.dirichlet] = 0.0
    op = O.make_operator(om, k, "scaled", modification=True)
    ref = op.residual(f, u)
    r = ctx.vector(level)
    nrm = ctx.residual(level, ctx.from_canonical(level, _dev(f)), ctx.from_canonical(level, _dev(u)), r, norm=True)
    got = ctx.to_canonical(level, r).cpu().numpy()
    assert _rel(got, ref) <= TOL64
    assert nrm == pytest.approx(np.linalg.norm(ref[om.unknowns]), rel=1e-13)


@pytest.mark.parametrize("mesh_fn,level,eta", [(flat_tet, 3, 100.0), (flat_tet, 4, 1000.0), (unit_tet, 4, 100.0)])
def test_modification_apply_matches_oracle(mesh_fn, level, eta):
    """Sec. 4.1 modification (3D reading): same triggered edges, same operator."""
    om, k, u, ctx = _setup(mesh_fn, level, kfun=lambda x: sigmoid_k(x, eta))
    mods, info = O.modification_factors(om, k)
    assert ctx.level_info(level)["n_modified"] == info["n_triggered"] > 0
    y = ctx.vector(level)
    ctx.apply_scaled(level, ctx.from_canonical(level, _dev(u)), y)
    got = ctx.to_canonical(level, y).cpu().numpy()
    ref = O.make_operator(om, k, "scaled", modification=True).apply(u)
    assert _rel(got, ref) <= TOL64 and _elem(got, ref) <= TOL64


@pytest.mark.parametrize("mesh_fn,level", [(kuhn_cube, 4), (unit_tet, 5), (kuhn_cube_2x2x2, 3)])
def test_chebyshev_bound_and_smoothing(mesh_fn, level):
    om, k, u, ctx = _setup(mesh_fn, level)
    op = O.make_operator(om, k, "scaled", modification=True)
    lam = O.gershgorin_lambda(op)
    assert ctx.level_info(level)["lambda_max"] == pytest.approx(lam, rel=1e-13)
    f = uniform_vector(om.n_nodes, seed=3)
    f[om.dirichlet] = 0.0
    ref = O.chebyshev(op, f, u, 3, lam)
    ud = ctx.from_canonical(level, _dev(u))
    ctx.smooth(level, ctx.from_canonical(level, _dev(f)), ud, 3, hhg.CHEBYSHEV)
    assert _rel(ctx.to_canonical(level, ud).cpu().numpy(), ref) <= 1e-11


@pytest.mark.parametrize("mesh_fn,level,coarse", [(kuhn_cube, 4, 2), (unit_tet, 6, 3), (kuhn_cube_2x2x2, 3, 1),
                                                   (regular_tet, 5, 3)])
def test_vcycle_fp64_matches_oracle(mesh_fn, level, coarse):
    X, T = mesh_fn()
    mg = O.Multigrid(X, T, level, coarse, kfun=smooth_k, modification=True)
    om = mg.meshes[level]
    ctx = hhg.Context(X, T, level)
    ctx.set_coefficient(smooth_k(om.xyz))
    ctx.set_coarse_level(coarse)
    f = uniform_vector(om.n_nodes, seed=11)
    f[om.dirichlet] = 0.0
    u = np.zeros(om.n_nodes)
    fd = ctx.from_canonical(level, _dev(f))
    ud = ctx.from_canonical(level, _dev(u))
    for it in range(3):
        u = mg.vcycle(level, f, u)
        ctx.vcycle(level, fd, ud, 2, 2, hhg.CHEBYSHEV)
        got = ctx.to_canonical(level, ud).cpu().numpy()
        assert _rel(got, u) <= 1e-11, (it, _rel(got, u))


@pytest.mark.parametrize("mesh_fn,level,coarse,eta,pre,post", [(flat_tet, 4, 2, 100.0, 2, 2),
                                                              (unit_tet, 5, 2, 100.0, 3, 1),
                                                              (kuhn_cube, 4, 2, None, 1, 3)])
def test_vcycle_smoother_sweeps_and_modification(mesh_fn, level, coarse, eta, pre, post):
    """V-cycles whose Chebyshev sweeps run with the Sec. 4.1 modification
    triggered (steep sigmoid k) and with odd sweep counts, against the
    oracle's V-cycle."""
    X, T = mesh_fn()
    kfun = smooth_k if eta is None else (lambda x: sigmoid_k(x, eta))
    mg = O.Multigrid(X, T, level, coarse, kfun=kfun, modification=True)
    om = mg.meshes[level]
    ctx = hhg.Context(X, T, level)
    ctx.set_coefficient(kfun(om.xyz))
    ctx.set_coarse_level(coarse)
    if eta is not None:
        assert sum(ctx.level_info(l)["n_modified"] for l in range(coarse + 1, level + 1)) > 0
    f = uniform_vector(om.n_nodes, seed=12)
    f[om.dirichlet] = 0.0
    u = np.zeros(om.n_nodes)
    fd = ctx.from_canonical(level, _dev(f))
    ud = ctx.from_canonical(level, _dev(u))
    for it in range(2):
        u = mg.vcycle(level, f, u, pre=pre, post=post)
        ctx.vcycle(level, fd, ud, pre, post, hhg.CHEBYSHEV)
        got = ctx.to_canonical(level, ud).cpu().numpy()
        assert _rel(got, u) <= 1e-11, (it, _rel(got, u))


@pytest.mark.parametrize("mesh_fn,level,coarse", [(kuhn_cube_2x2x2, 4, 1), (cube12, 4, 2), (flat_tet, 4, 2)])
def test_geometric_coarse_coefficients_match_oracle(mesh_fn, level, coarse):
    """HHG_FLAG_COARSE_K_GEOMETRIC: the coarse levels' operators (their k the
    geometric full-weighting averages of the finer level's) and two V(2,2)
    cycles against the oracle's multigrid with coarse_k="geometric"."""
    X, T = mesh_fn()
    kfun = lambda x: lognormal_k(x, lognormal_params(2, 1.5, 0.1))
    mg = O.Multigrid(X, T, level, coarse, kfun=kfun, modification=True, coarse_k="geometric")
    om = mg.meshes[level]
    ctx = hhg.Context(X, T, level, hhg.FLAG_COARSE_K_GEOMETRIC)
    ctx.set_coefficient(kfun(om.xyz))
    ctx.set_coarse_level(coarse)
    print(f"case {mesh_fn.__name__} level {level}", flush=True)
    for l in range(coarse, level):
        m = mg.meshes[l]
        v = uniform_vector(m.n_nodes, seed=l)
        v[m.dirichlet] = 0.0
        y = ctx.vector(l)
        ctx.apply_scaled(l, ctx.from_canonical(l, _dev(v)), y)
        got = ctx.to_canonical(l, y).cpu().numpy()
        ref = mg.ops[l].apply(v)
        assert _rel(got, ref) <= TOL64 and _elem(got, ref) <= TOL64, (l, _rel(got, ref))
    f = uniform_vector(om.n_nodes, seed=13)
    f[om.dirichlet] = 0.0
    u = np.zeros(om.n_nodes)
    fd = ctx.from_canonical(level, _dev(f))
    ud = ctx.from_canonical(level, _dev(u))
    for it in range(2):
        u = mg.vcycle(level, f, u)
        ctx.vcycle(level, fd, ud, 2, 2, hhg.CHEBYSHEV)
        got = ctx.to_canonical(level, ud).cpu().numpy()
        assert _rel(got, u) <= 1e-11, (it, _rel(got, u))


def test_device_coarse_inverse_matches_dense_solve():
    """Coarse levels above 512 unknowns are inverted on the device
    (Gauss-Jordan with partial pivoting): the 6-tet cube's level 4 (3375
    unknowns) as the coarse level, its solve against numpy's dense solve of
    the oracle's matrix (with the modification), and a V(2,2) cycle from
    level 5 against the oracle's cycle with the same coarse level."""
    X, T = kuhn_cube()
    level, coarse = 5, 4
    kfun = lambda x: lognormal_k(x, lognormal_params(6, 1.0, 0.15))
    mg = O.Multigrid(X, T, level, coarse, kfun=kfun, modification=True)
    ctx = hhg.Context(X, T, level)
    ctx.set_coefficient(kfun(mg.meshes[level].xyz))
    ctx.set_coarse_level(coarse)
    mc = mg.meshes[coarse]
    assert len(mc.unknowns) == 3375
    f = uniform_vector(mc.n_nodes, seed=31)
    f[mc.dirichlet] = 0.0
    uc = ctx.vector(coarse)
    ctx.vcycle(coarse, ctx.from_canonical(coarse, _dev(f)), uc, 2, 2, hhg.CHEBYSHEV)
    got = ctx.to_canonical(coarse, uc).cpu().numpy()
    ref = mg.coarse_solve(f)
    assert _rel(got, ref) <= 1e-11, _rel(got, ref)
    om = mg.meshes[level]
    f = uniform_vector(om.n_nodes, seed=32)
    f[om.dirichlet] = 0.0
    ud = ctx.vector(level)
    ctx.vcycle(level, ctx.from_canonical(level, _dev(f)), ud, 2, 2, hhg.CHEBYSHEV)
    ref = mg.vcycle(level, f, np.zeros(om.n_nodes))
    got = ctx.to_canonical(level, ud).cpu().numpy()
    assert _rel(got, ref) <= 1e-11, _rel(got, ref)


def test_geometric_coarse_coefficients_contract_faster_on_rough_k():
    """On the 48-tet cube with the rough lognormal field (sigma 1.5,
    correlation length 0.05), geometric coarse coefficients need fewer cycles
    to 1e-8 than sampled ones."""
    X, T = kuhn_cube_2x2x2()
    level = 5
    its = {}
    for name, flags in (("sample", 0), ("geometric", hhg.FLAG_COARSE_K_GEOMETRIC)):
        ctx = hhg.Context(X, T, level, flags)
        xyz, dirichlet = ctx.node_coords(level)
        prm = lognormal_params(2, 1.5, 0.05)
        ctx.set_coefficient(lognormal_k(xyz, prm))
        f = prm["rng"].uniform(-1, 1, len(xyz))
        f[dirichlet] = 0.0
        u = ctx.vector(level)
        st = ctx.solve(level, ctx.from_canonical(level, _dev(f)), u, mode=hhg.SOLVE_MIXED, tol=1e-8, max_iter=100)
        print(name, st, flush=True)
        assert st["rel_residual"] <= 1e-8
        its[name] = st["iterations"]
    assert its["geometric"] < its["sample"]


@pytest.mark.parametrize("mode", [hhg.SOLVE_F64, hhg.SOLVE_MIXED])
def test_solve_reaches_tolerance_and_oracle_solution(mode):
    X, T = kuhn_cube()
    level = 5
    om = O.Mesh(X, T, level)
    kfun = lambda x: lognormal_k(x, lognormal_params(2, 1.0, 0.2))
    k = kfun(om.xyz)
    ctx = hhg.Context(X, T, level)
    ctx.set_coefficient(k)
    f = uniform_vector(om.n_nodes, seed=5)
    f[om.dirichlet] = 0.0
    fd = ctx.from_canonical(level, _dev(f))
    ud = ctx.vector(level)
    st = ctx.solve(level, fd, ud, mode=mode, tol=1e-10, max_iter=60)
    assert st["rel_residual"] <= 1e-10, st
    import scipy.sparse.linalg as spla
    op = O.make_operator(om, k, "scaled", modification=True)
    ref = np.zeros(om.n_nodes)
    ref[om.unknowns] = spla.spsolve(op.A.tocsc(), f[om.unknowns])
    got = ctx.to_canonical(level, ud).cpu().numpy()
    assert _rel(got, ref) <= 1e-8, _rel(got, ref)


def test_solve_stops_on_a_non_finite_residual():
    """A NaN in the right-hand side gives a NaN residual norm, which ends the
    solve and is reported as such (not as a zero residual)."""
    om, k, u, ctx = _setup(kuhn_cube, 4)
    f = uniform_vector(om.n_nodes, seed=2)
    f[om.dirichlet] = 0.0
    f[om.unknowns[len(om.unknowns) // 2]] = np.nan
    fd = ctx.from_canonical(4, _dev(f))
    r = ctx.vector(4)
    assert np.isnan(ctx.residual(4, fd, ctx.vector(4), r, norm=True))
    for mode in (hhg.SOLVE_F64, hhg.SOLVE_MIXED):
        st = ctx.solve(4, fd, ctx.vector(4), mode=mode, tol=1e-8, max_iter=20)
        assert np.isnan(st["rel_residual"]) and st["iterations"] == 0, st


def test_c2_full_size_sampled_rows():
    """Unit tet level 8 (2.86M nodes), lognormal k (sigma 1, l_c 0.1, seed 1),
    u from the same stream: 400 sampled rows of the scaled and nodal applies
    against the oracle's row-by-row evaluation, plus properties that hold at
    any size (constant input -> zero interior rows for both operators)."""
    X, T = unit_tet()
    level = 8
    ctx = hhg.Context(X, T, level)
    om = O.Mesh(X, T, level)
    prm = lognormal_params(1, 1.0, 0.1)
    k = lognormal_k(om.xyz, prm)
    u = prm["rng"].uniform(-1, 1, om.n_nodes)
    u[om.dirichlet] = 0.0
    ctx.set_coefficient(k)
    ud = ctx.from_canonical(level, _dev(u))
    rng = np.random.default_rng(123)
    nodes = rng.choice(om.n_nodes, 400, replace=False)
    for kind in ("scaled", "nodal"):
        y = ctx.vector(level)
        (ctx.apply_scaled if kind == "scaled" else ctx.apply_nodal)(level, ud, y)
        got = ctx.to_canonical(level, y).cpu().numpy()
        ref = O.apply_rows(om, k, u, nodes, kind)
        scale = np.abs(ref).max()
        assert np.abs(got[nodes] - ref).max() <= TOL64 * scale, kind
        assert np.all(got[om.dirichlet] == 0.0)
    # FP32 applies (the bench's FP32 configuration) on the same rows, against
    # the oracle on the FP32-rounded u and k: FP32 arithmetic only
    u32 = u.astype(np.float32).astype(np.float64)
    k32 = k.astype(np.float32).astype(np.float64)
    ud32 = ctx.from_canonical(level, _dev(u32).float())
    for kind in ("scaled", "nodal"):
        y = ctx.vector(level, torch.float32)
        (ctx.apply_scaled if kind == "scaled" else ctx.apply_nodal)(level, ud32, y)
        got = ctx.to_canonical(level, y).cpu().numpy().astype(np.float64)
        ref = O.apply_rows(om, k32, u32, nodes, kind)
        scale = np.abs(ref).max()
        err = np.abs(got[nodes] - ref).max() / scale
        print(f"C2 FP32 {kind}: max sampled-row error {err:.2e} of the largest row", flush=True)
        assert err <= 2e-6, kind
        assert np.all(got[om.dirichlet] == 0.0)
    assert ctx.level_info(level)["n_modified"] == 0
    one = ctx.from_canonical(level, _dev(np.where(om.dirichlet, 0.0, 1.0)))
    interior = ~om.dirichlet & ~_touches_boundary(om)
    for fn in (ctx.apply_scaled, ctx.apply_nodal):
        y = ctx.vector(level)
        fn(level, one, y)
        v = ctx.to_canonical(level, y).cpu().numpy()
        assert np.abs(v[interior]).max() <= 1e-13 * np.abs(v).max()


def _touches_boundary(om):
    """Nodes with a Dirichlet neighbour (their rows see the zero boundary)."""
    n = 2 ** om.level
    lo = 1.5 / n
    x = om.xyz
    return (x.min(axis=1) < lo) | (x.sum(axis=1) > 1 - lo)


@pytest.mark.parametrize("case", ["scaled", "nodal", "mixed", "tensor"])
def test_graph_cycles_match_eager_cycles(case):
    """Solve-loop V-cycles replayed from captured HIP graphs give the same
    iterates, bit for bit, as eager cycles: many replays per solve with eager
    residual norms between them, a second solve on the same captures, and a
    new coefficient between (which must start new captures)."""
    X, T = cube12()
    level = 5
    om, _, _, ctx = _setup(cube12, level, kfun=smooth_k)
    f = uniform_vector(om.n_nodes, seed=9)
    f[om.dirichlet] = 0.0
    fd = ctx.from_canonical(level, _dev(f))
    mask = hhg.PRIM_VERTICES | hhg.PRIM_EDGES

    def solve(mode):
        u = ctx.vector(level)
        if case == "tensor":
            st = ctx.solve_tensor(level, fd, u, mode=mode, tol=1e-10, max_iter=60, pre=3, post=3)
        else:
            st = ctx.solve_form(level, fd, u, form=case, nodal_primitives=mask, mode=mode, tol=1e-10, max_iter=60,
                                pre=3, post=3)
        assert st["status"] == 0 and st["rel_residual"] <= 1e-10
        return st["iterations"], u

    for kfun in (smooth_k, lambda x: lognormal_k(x, lognormal_params(4, 1.0, 0.2))):
        k = kfun(om.xyz)
        ctx.set_coefficient(k)
        if case == "tensor":
            ctx.set_tensor_coefficient(tensor_fields(k[:, None, None] * tensor_K(om.xyz)))
        for mode in (hhg.SOLVE_F64, hhg.SOLVE_MIXED):
            ctx.set_graphs(True)
            n1, u1 = solve(mode)
            n2, u2 = solve(mode)
            ctx.set_graphs(False)
            n3, u3 = solve(mode)
            assert n1 == n2 == n3, (n1, n2, n3)
            assert torch.equal(u1, u3) and torch.equal(u2, u3)
