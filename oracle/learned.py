"""CPU reference of the learned smoothing correction (test infrastructure only).

The paper has no learned component; this module defines the network the
product's correction kernels must reproduce, written independently of them.

Per interior node i of a macro tet (nodes on macro faces/edges/vertices and
Dirichlet nodes get c = 0), with the 15 lattice positions p = 0 (the node) and
p = 1..14 the neighbours along the tet-local lattice directions
(1,0,0),(0,1,0),(0,0,1),(1,-1,0),(1,0,-1),(0,1,-1),(1,-1,1) and their
negatives, in that order:
    s_i  = max_p |r_p| + 1e-30                                   (float32)
    x_p  = r_p * fl32(1 / s_i),  x_{15+p} = L_p - L_0,  x_30 = x_31 = 0    (float32)
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
    inv = (np.float32(1.0) / s).astype(np.float32)  # one FP32 reciprocal per node
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
