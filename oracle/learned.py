"""CPU reference of the learned smoothing correction (test infrastructure only).

The paper has no learned component; this module defines the network the
product's correction kernels must reproduce, written independently of them.

Per interior node i of a macro tet (nodes on macro faces/edges/vertices and
Dirichlet nodes get c = 0), with the 15 lattice positions p = 0 (the node) and
p = 1..14 the neighbours along the tet-local lattice directions
(1,0,0),(0,1,0),(0,0,1),(1,-1,0),(1,0,-1),(0,1,-1),(1,-1,1) and their
negatives, in that order:
    s_i  = max_p |r_p| + 1e-30                                   (float32)
    x_p  = r_p * fl32(1 / s_i),  x_{15+p} = L_p - L_0,  x_30 = x_31 = 0
           (float32: the reciprocal rounded once, each product rounded once)
           with L = float32(log k) (log taken in float64)
    h1   = bf16(relu(float32(W1 bf16(x)) + b1))
    h2   = relu(float32(W2 h1) + b2)
    c    = float32(w3 . h2 + b3)
All parameters are BF16-valued (the float32 master copy rounded to nearest
even).  Matrix products are taken exactly here (float64) and rounded once to
float32, which the kernels' float32 accumulation matches up to its own
rounding order.

Parameter vector layout (817): W1[16][32], b1[16], W2[16][16], b2[16], w3[16], b3.
"""
import numpy as np

NPARAM = 16 * 32 + 16 + 16 * 16 + 16 + 16 + 1
DIRS = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, -1, 0), (1, 0, -1), (0, 1, -1), (1, -1, 1),
        (-1, 0, 0), (0, -1, 0), (0, 0, -1), (-1, 1, 0), (-1, 0, 1), (0, -1, 1), (-1, 1, -1)]


def bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out)


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    W1 = w[o:o + 512].reshape(16, 32); o += 512
    b1 = w[o:o + 16]; o += 16
    W2 = w[o:o + 256].reshape(16, 16); o += 256
    b2 = w[o:o + 16]; o += 16
    w3 = w[o:o + 16]; o += 16
    b3 = w[o]
    return W1, b1, W2, b2, w3, b3


def init_weights(seed=0):
    """Glorot-uniform FP32 master weights, zero biases, zero output layer
    (the correction starts at 0, i.e. the plain smoother)."""
    rng = np.random.default_rng(seed)
    w = np.zeros(NPARAM, dtype=np.float32)
    a1 = np.sqrt(6.0 / (32 + 16))
    w[:512] = rng.uniform(-a1, a1, 512)
    a2 = np.sqrt(6.0 / (16 + 16))
    w[528:784] = rng.uniform(-a2, a2, 256)
    return w


def stencil_positions(mesh, nodes):
    """For each node (interior of a macro tet), the canonical indices of the 15
    positions (the node, then the 14 directions) found from the node
    coordinates in the tet's own lattice frame."""
    n = 2 ** mesh.level
    per = (n - 1) * (n - 2) * (n - 3) // 6
    first = mesh.n_nodes - per * mesh.T.shape[0]
    out = np.empty((len(nodes), 15), dtype=np.int64)
    # lattice coordinates -> canonical index inside each tet (interior order k, j, i)
    for q, c in enumerate(nodes):
        t = (c - first) // per
        X = mesh.X[mesh.T[t]]
        E = np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], axis=1)
        lat = np.rint(np.linalg.solve(E, mesh.xyz[c] - X[0]) * n).astype(int)
        out[q, 0] = c
        for p, d in enumerate(DIRS):
            target = X[0] + E @ ((lat + np.array(d)) / n)
            j = _find(mesh, target)
            out[q, p + 1] = j
    return out


_cache = {}


def _find(mesh, x):
    key = id(mesh)
    if key not in _cache:
        from scipy.spatial import cKDTree
        _cache.clear()
        _cache[key] = cKDTree(mesh.xyz)
    d, j = _cache[key].query(x)
    assert d < 1e-9
    return int(j)


def interior_nodes(mesh):
    n = 2 ** mesh.level
    per = (n - 1) * (n - 2) * (n - 3) // 6
    return np.arange(mesh.n_nodes - per * mesh.T.shape[0], mesh.n_nodes)


def features(r32, logk32, pos):
    """(nodes, 32) float32 features and the scales s (float32)."""
    rp = r32[pos].astype(np.float32)
    s = (np.abs(rp).max(axis=1) + np.float32(1e-30)).astype(np.float32)
    x = np.zeros((pos.shape[0], 32), dtype=np.float32)
    inv = (np.float32(1.0) / s).astype(np.float32)   # one reciprocal per node
    x[:, :15] = rp * inv[:, None]
    lk = logk32[pos]
    x[:, 15:30] = lk - lk[:, :1]
    return x, s


def forward(w, x, round_activations=True):
    """c (float32), and the intermediates for backward."""
    W1, b1, W2, b2, w3, b3 = unpack(bf16(w) if round_activations else w)
    xb = bf16(x).astype(np.float64) if round_activations else x.astype(np.float64)
    z1 = (xb @ W1.T).astype(np.float32) + b1.astype(np.float32) if round_activations else xb @ W1.T + b1
    a1 = np.maximum(z1, 0)
    h1 = bf16(a1).astype(np.float64) if round_activations else a1.astype(np.float64)
    z2 = (h1 @ W2.T).astype(np.float32) + b2.astype(np.float32) if round_activations else h1 @ W2.T + b2
    h2 = np.maximum(z2, 0).astype(np.float64)
    c = h2 @ w3 + b3
    if round_activations:
        c = c.astype(np.float32)
    return c, dict(xb=xb, z1=np.asarray(z1, np.float64), h1=h1, z2=np.asarray(z2, np.float64), h2=h2)


def backward(w, cache, g, round_weights=True):
    """Gradient of sum_i g_i c_i with respect to the 817 parameters (float64);
    the BF16 roundings of x and h1 count as identities."""
    W1, b1, W2, b2, w3, b3 = unpack(bf16(w) if round_weights else w)
    g = np.asarray(g, dtype=np.float64)
    h2, h1, xb = cache["h2"], cache["h1"], cache["xb"]
    dw3 = h2.T @ g
    db3 = g.sum()
    dz2 = (g[:, None] * w3[None, :]) * (cache["z2"] > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (cache["z1"] > 0)
    dW1 = dz1.T @ xb
    db1 = dz1.sum(axis=0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, [db3]])


def correction(w, r, logk32, pos, nodes, n_nodes, round_activations=True):
    """s_i c_i on every node (0 off the interior nodes `nodes`), with the
    features taken from r rounded to float32; also the scales and the
    network's intermediates."""
    x, s = features(np.asarray(r, dtype=np.float32), logk32, pos)
    c, cache = forward(w, x, round_activations)
    sc = np.zeros(n_nodes)
    sc[nodes] = s.astype(np.float64) * np.asarray(c, dtype=np.float64)
    return sc, s, cache


def step(op, w, f, u, logk32, pos, nodes, omega=2.0 / 3.0):
    """One learned smoothing step on the unknowns:
        r = f - A u,   u <- u + D^{-1} (omega r + s c(r, k)),
    i.e. a damped Jacobi step plus the network's correction s c scaled by the
    inverse diagonal (c = 0 off the macro-tet interiors)."""
    r = op.residual(f, u)
    sc, _, _ = correction(w, r, logk32, pos, nodes, op.mesh.n_nodes)
    out = u.copy()
    idx = op.mesh.unknowns
    out[idx] += (omega * r[idx] + sc[idx]) / op.diag
    out[op.mesh.dirichlet] = 0.0
    return out


def loss_and_grad(op, w, r, e, logk32, pos, nodes, omega=2.0 / 3.0, round_activations=True):
    """Training loss of one sample (r, e) and its gradient in the parameters.

    e1 = e - D^{-1}(omega r + s c) is the error left after one learned step
    from an iterate with error e and residual r = A e;  L = e1'A e1 / e'A e
    (energy norms over the unknowns).  With A symmetric,
        dL/dc_i = -2 (A e1)_i s_i / (D_i e'A e)
    on the interior nodes, and dL/dw follows through backward()."""
    sc, s, cache = correction(w, r, logk32, pos, nodes, op.mesh.n_nodes, round_activations)
    idx = op.mesh.unknowns
    e1 = np.zeros(op.mesh.n_nodes)
    e1[idx] = e[idx] - (omega * r[idx] + sc[idx]) / op.diag
    ae1 = op.apply(e1)
    e0 = float(e[idx] @ op.apply(e)[idx])
    loss = float(e1[idx] @ ae1[idx]) / e0
    dinv = np.zeros(op.mesh.n_nodes)
    dinv[idx] = 1.0 / op.diag
    g = -2.0 * ae1[nodes] * s.astype(np.float64) * dinv[nodes] / e0
    return loss, backward(w, cache, g, round_weights=round_activations)


def vcycle(mg, w, f, u, logk32, pos, nodes, pre=2, post=2, omega=2.0 / 3.0):
    """One V(pre,post) cycle of the oracle's multigrid (Multigrid in
    oracle.py) whose finest level smooths with learned steps; the coarser
    levels keep Chebyshev smoothing.  logk32, pos, nodes belong to the finest
    level."""
    L = mg.levels[-1]
    op = mg.ops[L]
    for _ in range(pre):
        u = step(op, w, f, u, logk32, pos, nodes, omega)
    r = op.residual(f, u)
    mc = mg.meshes[L - 1]
    fc = mg.P[L].T @ r
    fc[mc.dirichlet] = 0.0
    uc = mg.vcycle(L - 1, fc, np.zeros(mc.n_nodes), pre, post)
    u = u + mg.P[L] @ uc
    u[op.mesh.dirichlet] = 0.0
    for _ in range(post):
        u = step(op, w, f, u, logk32, pos, nodes, omega)
    return u
