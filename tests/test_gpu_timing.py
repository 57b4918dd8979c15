"""The apply-timing instrumentation (hhg_set_timing / hhg_read_timing).

The events are stamped by the stencil launches themselves, so the window of
one timed apply lies inside a pair of events recorded on the same stream
around the call.  Timing changes no result: timed applies are bit-identical
to untimed ones, on a single tet (one interior kernel) and on the Kuhn cube
(interior kernel and inter-tet rows), in FP64 and FP32.
"""
import numpy as np
import pytest

from hhg_inputs import unit_tet, kuhn_cube, smooth_k, uniform_vector

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1709_06793_amd import hhg  # noqa: E402


@pytest.mark.parametrize("mesh_fn,level", [(unit_tet, 6), (kuhn_cube, 5)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_timed_applies_lie_inside_the_calls_and_change_nothing(mesh_fn, level, dtype):
    print(f"case {mesh_fn.__name__} level {level} {dtype}", flush=True)
    X, T = mesh_fn()
    ctx = hhg.Context(X, T, level)
    xyz, dirichlet = ctx.node_coords(level)
    ctx.set_coefficient(smooth_k(xyz))
    u = uniform_vector(len(xyz), seed=3)
    u[dirichlet] = 0.0
    uv = ctx.from_canonical(level, torch.tensor(u, device="cuda")).to(dtype)
    y0 = ctx.vector(level, dtype)
    ctx.apply_scaled(level, uv, y0)
    torch.cuda.synchronize()

    y1 = ctx.vector(level, dtype)
    reps = 5
    outer = []
    ctx.set_timing(True)
    inner = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        ctx.apply_scaled(level, uv, y1)
        b.record()
        torch.cuda.synchronize()
        outer.append(a.elapsed_time(b))
        ms, n = ctx.read_timing()
        assert n == 1
        inner.append(ms)
    ctx.set_timing(False)
    assert ctx.read_timing() == (0.0, 0)
    for t_in, t_out in zip(inner, outer):
        assert np.isfinite(t_in) and t_in > 0.0
        assert t_in <= t_out + 2e-3, (t_in, t_out)  # 2 us for the two clocks' rounding
    assert torch.equal(y0, y1)


def test_calls_go_to_torchs_current_stream():
    """The binding passes the handle of torch's current stream (default
    priority side stream here): an apply issued inside `torch.cuda.stream`
    runs there and gives the default stream's result."""
    X, T = kuhn_cube()
    level = 4
    ctx = hhg.Context(X, T, level)
    xyz, dirichlet = ctx.node_coords(level)
    ctx.set_coefficient(smooth_k(xyz))
    u = uniform_vector(len(xyz), seed=4)
    u[dirichlet] = 0.0
    uv = ctx.from_canonical(level, torch.tensor(u, device="cuda"))
    y0, y1 = ctx.vector(level), ctx.vector(level)
    assert (hhg._stream().value or 0) == torch.cuda.current_stream().cuda_stream
    ctx.apply_scaled(level, uv, y0)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        assert (hhg._stream().value or 0) == s.cuda_stream != torch.cuda.default_stream().cuda_stream
        ctx.apply_scaled(level, uv, y1)
    s.synchronize()
    assert torch.equal(y0, y1)
