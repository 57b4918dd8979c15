"""Pins of the learned-correction reference (CPU): BF16 rounding against exact
bit patterns, the analytic gradient against central differences, and the
zero-output start."""
import numpy as np
import pytest

from oracle import learned as LN


def test_bf16_rounding_bit_patterns():
    u = np.array([0x3F800000, 0x3F808000, 0x3F818000, 0x3F808001, 0xBF7FFFFF, 0x00000001], dtype=np.uint32)
    want = np.array([0x3F800000, 0x3F800000, 0x3F820000, 0x3F810000, 0xBF800000, 0x00000000], dtype=np.uint32)
    got = LN.bf16(u.view(np.float32)).view(np.uint32)
    assert np.array_equal(got, want)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    w = rng.normal(0, 0.4, LN.NPARAM)
    x = rng.normal(0, 1, (40, 32))
    g = rng.normal(0, 1, 40)
    c, cache = LN.forward(w, x, round_activations=False)
    grad = LN.backward(w, cache, g, round_weights=False)
    f = lambda ww: float(g @ LN.forward(ww, x, round_activations=False)[0])
    h = 1e-6
    idx = rng.choice(LN.NPARAM, 60, replace=False)
    idx = np.union1d(idx, [0, 511, 512, 527, 528, 783, 784, 799, 800, 815, 816])
    for p in idx:
        e = np.zeros(LN.NPARAM)
        e[p] = h
        fd = (f(w + e) - f(w - e)) / (2 * h)
        assert fd == pytest.approx(grad[p], rel=1e-6, abs=1e-7), p


def test_zero_output_layer_gives_zero_correction():
    w = LN.init_weights(0)
    x = np.random.default_rng(1).normal(0, 1, (10, 32)).astype(np.float32)
    c, _ = LN.forward(w, x)
    assert np.all(c == 0)


def test_stencil_positions_worked_by_hand():
    """The unit tet at level 2 has one interior node, (1,1,1)/4; its 15
    positions are that node and (1,1,1) + d for the 14 lattice directions in
    DIR order, at coordinates (lattice)/4.  On the regular tet the same
    lattice points map through x = v0 + (i(v1-v0) + j(v2-v0) + k(v3-v0))/4."""
    from oracle import oracle as O
    from hhg_inputs import unit_tet, regular_tet
    want_lat = np.array([(1, 1, 1), (2, 1, 1), (1, 2, 1), (1, 1, 2), (2, 0, 1), (2, 1, 0), (1, 2, 0),
                         (2, 0, 2), (0, 1, 1), (1, 0, 1), (1, 1, 0), (0, 2, 1), (0, 1, 2), (1, 0, 2),
                         (0, 2, 0)], dtype=np.float64)
    for fn in (unit_tet, regular_tet):
        X, T = fn()
        m = O.Mesh(X, T, 2)
        nodes = LN.interior_nodes(m)
        assert len(nodes) == 1
        pos = LN.stencil_positions(m, nodes)
        v = X[T[0]]
        want = v[0] + want_lat @ np.stack([v[1] - v[0], v[2] - v[0], v[3] - v[0]]) / 4.0
        assert np.abs(m.xyz[pos[0]] - want).max() < 1e-14


def test_features_worked_by_hand():
    """s = max |r| over the 15 positions (+1e-30), x_p = r_p * fl32(1/s) (one
    FP32 reciprocal per node, each product rounded once), x_{15+p} =
    log k_p - log k_0, x_30 = x_31 = 0."""
    r = np.zeros(20, dtype=np.float32)
    pos = np.arange(15)[None, :] + 2
    r[2:17] = [0.5, -2.0, 1.0, 0.25, 0, 0, 1.5, -0.75, 0, 0, 0, 0.125, 0, -1.0, 2.0]
    lk = np.zeros(20, dtype=np.float32)
    lk[2:17] = np.arange(15, dtype=np.float32) * 0.5 + 1.0
    x, s = LN.features(r, lk, pos)
    assert s[0] == np.float32(2.0)
    want = np.array([0.25, -1.0, 0.5, 0.125, 0, 0, 0.75, -0.375, 0, 0, 0, 0.0625, 0, -0.5, 1.0], dtype=np.float32)
    assert np.array_equal(x[0, :15], want)
    assert np.array_equal(x[0, 15:30], np.arange(15, dtype=np.float32) * 0.5)
    assert x[0, 30] == 0 and x[0, 31] == 0
    # s = 3: 1/3 rounds to 0x3EAAAAAB; 0.3 * that rounds differently from 0.3 / 3
    r2 = np.zeros(20, dtype=np.float32)
    r2[2] = np.float32(3.0)
    r2[3] = np.float32(0.3)
    x2, _ = LN.features(r2, lk, pos)
    inv = np.float32(1.0) / np.float32(3.0)
    assert inv.view(np.uint32) == 0x3EAAAAAB
    assert x2[0, 1] == np.float32(np.float64(np.float32(0.3)) * np.float64(inv))
    assert x2[0, 1] != np.float32(np.float64(np.float32(0.3)) / 3.0)
    assert x2[0, 0] == np.float32(1.0)


def test_loss_gradient_matches_central_differences():
    """dL/dw of the training loss (one learned step's remaining error energy
    relative to the initial one) through the oracle operator and backward(),
    against central differences of the loss of the unrounded network."""
    from oracle import oracle as O
    from hhg_inputs import kuhn_cube, smooth_k
    X, T = kuhn_cube()
    m = O.Mesh(X, T, 3)
    k = smooth_k(m.xyz) + 0.2
    op = O.make_operator(m, k, "scaled")
    nodes = LN.interior_nodes(m)
    pos = LN.stencil_positions(m, nodes)
    lk = np.log(k).astype(np.float32)
    rng = np.random.default_rng(11)
    e = rng.uniform(-1, 1, m.n_nodes)
    e[m.dirichlet] = 0.0
    r = op.apply(e)
    w = rng.normal(0, 0.3, LN.NPARAM)
    L0, g = LN.loss_and_grad(op, w, r, e, lk, pos, nodes, round_activations=False)
    assert 0 < L0
    f = lambda ww: LN.loss_and_grad(op, ww, r, e, lk, pos, nodes, round_activations=False)[0]
    h = 1e-6
    idx = np.union1d(rng.choice(LN.NPARAM, 40, replace=False), [0, 530, 790, 805, 816])
    for p in idx:
        d = np.zeros(LN.NPARAM)
        d[p] = h
        fd = (f(w + d) - f(w - d)) / (2 * h)
        assert fd == pytest.approx(g[p], rel=1e-5, abs=1e-8), p


def test_learned_step_with_zero_output_is_damped_jacobi():
    """A network with a zero output layer leaves the plain damped Jacobi step;
    a network with constant output b3 adds D^{-1} s b3 on interior nodes only."""
    from oracle import oracle as O
    from hhg_inputs import kuhn_cube, smooth_k
    X, T = kuhn_cube()
    m = O.Mesh(X, T, 3)
    k = smooth_k(m.xyz)
    op = O.make_operator(m, k, "scaled")
    nodes = LN.interior_nodes(m)
    pos = LN.stencil_positions(m, nodes)
    lk = np.log(k).astype(np.float32)
    rng = np.random.default_rng(2)
    f = rng.uniform(-1, 1, m.n_nodes)
    f[m.dirichlet] = 0
    u = rng.uniform(-1, 1, m.n_nodes)
    u[m.dirichlet] = 0
    w = LN.init_weights(0)
    got = LN.step(op, w, f, u, lk, pos, nodes)
    want = O.jacobi(op, f, u, 1)
    assert np.abs(got - want).max() < 1e-14
    w2 = w.copy()
    w2[816] = 0.5                                  # bf16-exact constant output
    got2 = LN.step(op, w2, f, u, lk, pos, nodes)
    rf = op.residual(f, u).astype(np.float32)
    s = np.abs(rf[pos]).max(axis=1) + np.float32(1e-30)
    dinv = np.zeros(m.n_nodes)
    dinv[m.unknowns] = 1.0 / op.diag
    delta = np.zeros(m.n_nodes)
    delta[nodes] = dinv[nodes] * s.astype(np.float64) * 0.5
    assert np.abs(got2 - want - delta).max() < 1e-14
