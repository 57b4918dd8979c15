"""Parity of the 2D HIP path (include/hhg2d.h) with the 2D oracle: stencil
scaling with and without the MA2 modification (Sec. 4.1) and nodal
integration, FP64 to 1e-12 of the largest entry, FP32 to a few 1e-6; the
number of replaced edge factors; properties at a large level."""
import numpy as np
import pytest

from hhg_inputs import obtuse_triangle, square_right4, square_nondelaunay8, sigmoid_k, smooth_k, uniform_vector
from oracle import oracle2d as O2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1709_06793_amd import hhg2d  # noqa: E402


def _match(ctx_xy, oracle_xy):
    """perm with ctx_xy[perm[q]] == oracle_xy[q] (coordinates agree to rounding)."""
    def order(xy):
        r = np.round(xy * 2 ** 20).astype(np.int64)
        return np.lexsort((r[:, 1], r[:, 0]))
    a, b = order(ctx_xy), order(oracle_xy)
    perm = np.empty(len(b), dtype=np.int64)
    perm[b] = a
    assert np.abs(ctx_xy[perm] - oracle_xy).max() <= 1e-12
    return perm


def _kfun(name):
    return {"sigmoid1000": lambda xy: sigmoid_k(xy, 1000.0), "sigmoid10": lambda xy: sigmoid_k(xy, 10.0),
            "smooth": lambda xy: smooth_k(np.c_[xy, np.full(len(xy), 0.3)])}[name]


@pytest.mark.parametrize("mesh_fn,level", [(obtuse_triangle, 4), (obtuse_triangle, 6), (square_right4, 3),
                                           (square_nondelaunay8, 1), (square_nondelaunay8, 3),
                                           (square_nondelaunay8, 5)])
@pytest.mark.parametrize("kname", ["sigmoid1000", "sigmoid10", "smooth"])
def test_2d_applies_match_oracle(mesh_fn, level, kname):
    X, T = mesh_fn()
    print(f"2D case {mesh_fn.__name__} level {level} k {kname}", flush=True)
    m = O2.Mesh2D(X, T, level)
    k = _kfun(kname)(m.xy)
    u = uniform_vector(m.n_nodes, seed=level)
    u[m.dirichlet] = 0.0
    for flags, mod in ((0, True), (hhg2d.FLAG_NO_MODIFICATION, False)):
        ctx = hhg2d.Context2D(X, T, level, flags)
        cxy, cdir = ctx.node_coords()
        assert len(cxy) == m.n_nodes
        perm = _match(cxy, m.xy)
        assert np.array_equal(cdir[perm], m.dirichlet)
        with pytest.raises(hhg2d.HHGError):
            ctx.apply_scaled(ctx.vector(), ctx.vector())
        kc = np.empty(m.n_nodes)
        kc[perm] = k
        ctx.set_coefficient(kc)
        mods, _ = O2.modification(m, k)
        assert ctx.sizes()["n_modified"] == (len(mods) if mod else 0)
        uc = np.empty(m.n_nodes)
        uc[perm] = u
        ud = ctx.from_canonical(torch.tensor(uc, device="cuda"))
        for kind, fn in (("scaled", ctx.apply_scaled), ("nodal", ctx.apply_nodal)):
            if kind == "nodal" and not mod:
                continue
            y = ctx.vector()
            fn(ud, y)
            got = ctx.to_canonical(y).cpu().numpy()[perm]
            ref = O2.apply(m, O2.assemble(m, k, kind, mod and kind == "scaled"), u)
            err = np.abs(got - ref).max() / np.abs(ref).max()
            assert err <= 1e-12, (kind, mod, err)
            assert np.all(got[m.dirichlet] == 0.0)
            y32 = ctx.vector(torch.float32)
            fn(ud.float(), y32)
            got32 = ctx.to_canonical(y32).cpu().numpy().astype(np.float64)[perm]
            assert np.abs(got32 - ref).max() / np.abs(ref).max() <= 4e-6, kind
        ctx.close()


def test_2d_large_level_properties():
    """Level 11 of the non-Delaunay square (16.8M nodes) with a sigmoid steep
    enough (m = 2000) that MA2 still replaces factors there: the operator
    stays symmetric (u.Av = v.Au to rounding), constants give zero rows away
    from the boundary, and copies of shared nodes agree."""
    X, T = square_nondelaunay8()
    level = 11
    ctx = hhg2d.Context2D(X, T, level)
    xy, dirichlet = ctx.node_coords()
    print(f"2D level {level}: {len(xy)} nodes", flush=True)
    k = sigmoid_k(xy, 1000.0, m=2000.0)
    ctx.set_coefficient(k)
    assert ctx.sizes()["n_modified"] > 0
    rng = np.random.default_rng(4)
    a = rng.uniform(-1, 1, len(xy))
    b = rng.uniform(-1, 1, len(xy))
    a[dirichlet] = 0.0
    b[dirichlet] = 0.0
    ad, bd = ctx.from_canonical(torch.tensor(a, device="cuda")), ctx.from_canonical(torch.tensor(b, device="cuda"))
    ya, yb = ctx.vector(), ctx.vector()
    ctx.apply_scaled(ad, ya)
    ctx.apply_scaled(bd, yb)
    ca, cb = ctx.to_canonical(ya).cpu().numpy(), ctx.to_canonical(yb).cpu().numpy()
    s1, s2 = float(b @ ca), float(a @ cb)
    assert abs(s1 - s2) <= 1e-10 * np.abs(ca).sum(), (s1, s2)
    # every copy holds the row value: slot vector equals the scatter of its canonical gather
    back = ctx.from_canonical(torch.tensor(ca, device="cuda"))
    assert torch.equal(back, ya)
    one = np.where(dirichlet, 0.0, 1.0)
    y1 = ctx.vector()
    ctx.apply_scaled(ctx.from_canonical(torch.tensor(one, device="cuda")), y1)
    v = ctx.to_canonical(y1).cpu().numpy()
    h = 0.5 / 2 ** level
    inner = (xy.min(axis=1) > 2 * h) & (xy.max(axis=1) < 1 - 2 * h)
    assert np.abs(v[inner]).max() <= 1e-12 * np.abs(v).max()


def test_2d_error_paths():
    """Bad coefficients and vectors are rejected with an error, not run."""
    X, T = square_nondelaunay8()
    ctx = hhg2d.Context2D(X, T, 3)
    xy, _ = ctx.node_coords()
    k = np.ones(len(xy))
    k[5] = -1.0
    with pytest.raises(hhg2d.HHGError):
        ctx.set_coefficient(k)
    k[5] = np.nan
    with pytest.raises(hhg2d.HHGError):
        ctx.set_coefficient(k)
    ctx.set_coefficient(np.ones(len(xy)))
    u = ctx.vector()
    with pytest.raises(hhg2d.HHGError):
        ctx.apply_scaled(u, u)
    with pytest.raises(hhg2d.HHGError):
        hhg2d.Context2D(X, np.array([[0, 1, 1]]), 3)
