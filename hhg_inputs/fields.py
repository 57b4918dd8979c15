"""Coefficient fields, manufactured solutions and seeded random vectors.

Every function takes node coordinates xyz (n, 3) and returns values there.
Random streams use NumPy's PCG64 (`numpy.random.default_rng(seed)`), drawn in
the order documented per function.
"""
import numpy as np


def smooth_k(xyz):
    """k = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z), in [0.5, 1.5]."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.sin(2 * np.pi * z)


def cosine_k(xyz, m):
    """k = cos(m pi x y z) + 2, in [1, 3] (the scalar coefficient of the
    paper's 3D scalar comparison, Sec. 7.2, with m = 3 or 8)."""
    return np.cos(m * np.pi * xyz[:, 0] * xyz[:, 1] * xyz[:, 2]) + 2.0


def affine_k(xyz, c=(2.0, 3.0, 5.0), c0=1.0):
    """k = 2x + 3y + 5z + 1 (the affine coefficient of the reproduction example)."""
    return c0 + xyz @ np.asarray(c, dtype=np.float64)


def sigmoid_k(xyz, eta, m=50.0):
    """k = eta / (1 + exp(-m (y - x - 0.2))) + 1, the steep coefficient the paper
    uses for its pre-asymptotic counter example, evaluated in 3D."""
    x, y = xyz[:, 0], xyz[:, 1]
    # exp's argument is capped where the quotient is below 1e-300 anyway
    return eta / (1.0 + np.exp(np.minimum(-m * (y - x - 0.2), 700.0))) + 1.0


def lognormal_params(seed, sigma=None, corr_len=None, modes=32):
    """Random Fourier modes of a Gaussian field with covariance
    sigma^2 exp(-|r|^2 / (2 corr_len^2)).  Draw order from default_rng(seed):
    [sigma ~ U(0.5, 2), corr_len ~ U(0.05, 0.3) when not given], omega
    (modes x 3, N(0, corr_len^-2)), phi (modes, U(0, 2 pi))."""
    rng = np.random.default_rng(seed)
    if sigma is None:
        sigma = rng.uniform(0.5, 2.0)
    if corr_len is None:
        corr_len = rng.uniform(0.05, 0.3)
    omega = rng.normal(0.0, 1.0 / corr_len, size=(modes, 3))
    phi = rng.uniform(0.0, 2 * np.pi, size=modes)
    return dict(sigma=float(sigma), corr_len=float(corr_len), omega=omega, phi=phi, rng=rng)


def lognormal_k(xyz, params, chunk=1 << 20):
    """k = exp(g), g = sigma sqrt(2/M) sum_m cos(omega_m . x + phi_m)."""
    om, ph, s = params["omega"], params["phi"], params["sigma"]
    M = om.shape[0]
    out = np.empty(xyz.shape[0])
    for a in range(0, xyz.shape[0], chunk):
        g = np.cos(xyz[a:a + chunk] @ om.T + ph).sum(axis=1)
        out[a:a + chunk] = np.exp(s * np.sqrt(2.0 / M) * g)
    return out


def lognormal_k_torch(xyz, params, torch, device="cuda", chunk=1 << 24):
    """lognormal_k evaluated with torch on `device` (same formula, FP64), for
    node sets too large for the numpy version; returns a device tensor."""
    x = torch.as_tensor(xyz, dtype=torch.float64, device=device)
    om = torch.tensor(params["omega"], dtype=torch.float64, device=device)
    ph = torch.tensor(params["phi"], dtype=torch.float64, device=device)
    g = torch.empty(x.shape[0], dtype=torch.float64, device=device)
    for a in range(0, x.shape[0], chunk):
        g[a:a + chunk] = torch.cos(x[a:a + chunk] @ om.T + ph).sum(dim=1)
    M = om.shape[0]
    return torch.exp(params["sigma"] * np.sqrt(2.0 / M) * g)


# directions c_m of the tensor operator's components D_m = c_m . grad
TENSOR_DIRS = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 0, 1], [0, 1, 1]], dtype=np.float64)


def tensor_K(xyz):
    """A smooth symmetric positive definite 3x3 field (n, 3, 3):
    K = s R diag(1, 1.5, 2.5) R^T, s = smooth_k, R the rotation about
    (1,1,1)/sqrt(3) by 0.8 sin(2 pi x) + 0.5 cos(2 pi z)."""
    n = xyz.shape[0]
    th = 0.8 * np.sin(2 * np.pi * xyz[:, 0]) + 0.5 * np.cos(2 * np.pi * xyz[:, 2])
    a = np.ones(3) / np.sqrt(3.0)
    A = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    R = (np.eye(3)[None] + np.sin(th)[:, None, None] * A[None]
         + (1 - np.cos(th))[:, None, None] * (A @ A)[None])
    D = np.diag([1.0, 1.5, 2.5])
    return smooth_k(xyz)[:, None, None] * (R @ D[None] @ np.transpose(R, (0, 2, 1)))


def tensor_fields(K):
    """The six coefficient fields (6, n) of K in the components D_m = c_m.grad
    (TENSOR_DIRS): k_i = K_ii - sum_{j != i} K_ij for D = d/dx_i, and
    k_ij = K_ij for D = d/dx_i + d/dx_j, so that
    sum_m k_m (c_m.a)(c_m.b) = a^T K b."""
    K = np.asarray(K, dtype=np.float64)
    out = np.empty((6, K.shape[0]))
    for i in range(3):
        out[i] = K[:, i, i] - sum(K[:, i, j] for j in range(3) if j != i)
    out[3], out[4], out[5] = K[:, 0, 1], K[:, 0, 2], K[:, 1, 2]
    return out


def tensor_fields_torch(xyz, torch, device="cuda", chunk=1 << 22):
    """tensor_fields(tensor_K(xyz)) evaluated with torch on `device` in
    chunks (same formulas, FP64); returns a (6, n) device tensor."""
    x = torch.as_tensor(xyz, dtype=torch.float64, device=device)
    n = x.shape[0]
    out = torch.empty((6, n), dtype=torch.float64, device=device)
    a = torch.ones(3, dtype=torch.float64, device=device) / np.sqrt(3.0)
    A = torch.tensor([[0.0, -a[2].item(), a[1].item()], [a[2].item(), 0.0, -a[0].item()],
                      [-a[1].item(), a[0].item(), 0.0]], dtype=torch.float64, device=device)
    D = torch.diag(torch.tensor([1.0, 1.5, 2.5], dtype=torch.float64, device=device))
    I3 = torch.eye(3, dtype=torch.float64, device=device)
    for c0 in range(0, n, chunk):
        xc = x[c0:c0 + chunk]
        th = 0.8 * torch.sin(2 * np.pi * xc[:, 0]) + 0.5 * torch.cos(2 * np.pi * xc[:, 2])
        R = I3[None] + torch.sin(th)[:, None, None] * A[None] + (1 - torch.cos(th))[:, None, None] * (A @ A)[None]
        s = 1.0 + 0.5 * torch.sin(2 * np.pi * xc[:, 0]) * torch.sin(2 * np.pi * xc[:, 1]) * torch.sin(2 * np.pi * xc[:, 2])
        K = s[:, None, None] * (R @ D[None] @ R.transpose(1, 2))
        for i in range(3):
            out[i, c0:c0 + chunk] = K[:, i, i] - sum(K[:, i, j] for j in range(3) if j != i)
        out[3, c0:c0 + chunk] = K[:, 0, 1]
        out[4, c0:c0 + chunk] = K[:, 0, 2]
        out[5, c0:c0 + chunk] = K[:, 1, 2]
    return out


def polynomial_tensor_K(xyz, lib=np):
    """The polynomial SPD permeability of the paper's tensor comparison
    (Sec. 7.3): diagonal x^2+2y^2+3z^2+1, 2x^2+3y^2+z^2+1, 3x^2+y^2+2z^2+1,
    off-diagonal K_xy = -y^2, K_xz = -z^2, K_yz = -x^2.  (n, 3, 3); `lib`
    numpy or torch (xyz of that library)."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    rows = [[x * x + 2 * y * y + 3 * z * z + 1, -y * y, -z * z],
            [-y * y, 2 * x * x + 3 * y * y + z * z + 1, -x * x],
            [-z * z, -x * x, 3 * x * x + y * y + 2 * z * z + 1]]
    return lib.stack([lib.stack(r, 1) for r in rows], 1)


def polynomial_tensor_fields_torch(xyz, torch, device="cuda", chunk=1 << 22):
    """tensor_fields(polynomial_tensor_K(xyz)) with torch on `device` in
    chunks (same formulas, FP64); returns a (6, n) device tensor."""
    x = torch.as_tensor(xyz, dtype=torch.float64, device=device)
    n = x.shape[0]
    out = torch.empty((6, n), dtype=torch.float64, device=device)
    for c0 in range(0, n, chunk):
        K = polynomial_tensor_K(x[c0:c0 + chunk], torch)
        for i in range(3):
            out[i, c0:c0 + chunk] = K[:, i, i] - sum(K[:, i, j] for j in range(3) if j != i)
        out[3, c0:c0 + chunk] = K[:, 0, 1]
        out[4, c0:c0 + chunk] = K[:, 0, 2]
        out[5, c0:c0 + chunk] = K[:, 1, 2]
    return out


def uniform_vector(n, seed=None, rng=None, lo=-1.0, hi=1.0):
    """n values uniform in [lo, hi) from default_rng(seed) (or a given stream)."""
    if rng is None:
        rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=n)


def manufactured_u(xyz):
    """u* = sin(pi x) sin(pi y) sin(pi z) (vanishes on the unit cube's boundary)."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    return np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def manufactured_f(xyz):
    """f = -div(k grad u*) for k = smooth_k and u* = manufactured_u."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    p = np.pi
    sx, sy, sz = np.sin(p * x), np.sin(p * y), np.sin(p * z)
    cx, cy, cz = np.cos(p * x), np.cos(p * y), np.cos(p * z)
    s2x, s2y, s2z = np.sin(2 * p * x), np.sin(2 * p * y), np.sin(2 * p * z)
    c2x, c2y, c2z = np.cos(2 * p * x), np.cos(2 * p * y), np.cos(2 * p * z)
    k = 1.0 + 0.5 * s2x * s2y * s2z
    gk = 0.5 * 2 * p * np.stack([c2x * s2y * s2z, s2x * c2y * s2z, s2x * s2y * c2z], axis=1)
    gu = p * np.stack([cx * sy * sz, sx * cy * sz, sx * sy * cz], axis=1)
    lap_u = -3 * p * p * sx * sy * sz
    return -(np.sum(gk * gu, axis=1) + k * lap_u)


def _freudenthal_mass_stencil():
    """Consistent P1 mass-matrix stencil of the Freudenthal triangulation of a
    grid of unit cubes (each cube cut into the 6 tetrahedra along the monotone
    paths from its lower to its upper corner), in units of the cube volume:
    {offset: sum over tets holding the origin and the offset of |t|/20
    (1 + delta)}, |t| = 1/6."""
    import itertools
    st = {}
    for c in itertools.product((-1, 0), repeat=3):
        for perm in itertools.permutations(range(3)):
            p = list(c)
            path = [tuple(p)]
            for ax in perm:
                p[ax] += 1
                path.append(tuple(p))
            if (0, 0, 0) not in path:
                continue
            for v in path:
                st[v] = st.get(v, 0.0) + (2.0 if v == (0, 0, 0) else 1.0) / 20.0 / 6.0
    return st


def kuhn_cube_mass_rhs(xyz, level, f):
    """b = M I_h f for the 6-tet Kuhn unit cube at `level` (the Freudenthal
    triangulation of the (2^level)^3 grid), at the nodes xyz (any order):
    f sampled on the grid, then the consistent mass stencil, h^3 per cube.
    Nodes on the boundary get the same formula (callers zero Dirichlet
    rows)."""
    n = 2 ** level
    g = np.arange(n + 1) / n
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    F = f(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)).reshape(n + 1, n + 1, n + 1)
    Fp = np.pad(F, 1)
    B = np.zeros_like(F)
    for (a, b, c), w in _freudenthal_mass_stencil().items():
        B += w * Fp[1 + a:n + 2 + a, 1 + b:n + 2 + b, 1 + c:n + 2 + c]
    idx = np.rint(np.asarray(xyz) * n).astype(np.int64)
    return B[idx[:, 0], idx[:, 1], idx[:, 2]] / float(n) ** 3


# ---------------------------------------------------------------- blending example
# The half cylinder mantle of Sec. 7.4 on its reference box (r1, r2) x (0, pi)
# x (0, z1), warped by w(z) = 0.2 sin(pi z / z1): with the mapping Phi from
# the physical to the reference domain, the Laplacian becomes -div(K grad u)
# with K = (D Phi)(D Phi)^T / |det D Phi| at x = Phi^{-1}(xh), here times the
# material parameter 1 + z.
CYL_R1, CYL_R2, CYL_Z1, CYL_WARP = 0.8, 1.0, 4.0, 0.2


def cylinder_warp(z, lib=np):
    """w(z), w'(z), w''(z) of the warp w(z) = 0.2 sin(pi z / z1)."""
    k = np.pi / CYL_Z1
    return CYL_WARP * lib.sin(k * z), CYL_WARP * k * lib.cos(k * z), -CYL_WARP * k * k * lib.sin(k * z)


def cylinder_mapping_K(xyz, lib=np):
    """K = (D Phi)(D Phi)^T / |det D Phi| at the reference points xyz (n, 3, 3):
    with r = x - w(z) the physical radius and p = w'(z),
    K = r [[p^2 + 1, 0, p], [0, 1 / r^2, 0], [p, 0, 1]]."""
    x, z = xyz[:, 0], xyz[:, 2]
    w, p, _ = cylinder_warp(z, lib)
    r = x - w
    zero = 0 * r
    rows = [[r * (p * p + 1), zero, r * p], [zero, 1 / r, zero], [r * p, zero, r]]
    return lib.stack([lib.stack(q, 1) for q in rows], 1)


def cylinder_phi_inverse(xyz):
    """Phi^{-1}: reference (radius + warp, angle, height) -> physical (x, y, z)."""
    w, _, _ = cylinder_warp(xyz[:, 2])
    r = xyz[:, 0] - w
    return np.stack([r * np.cos(xyz[:, 1]), r * np.sin(xyz[:, 1]), xyz[:, 2]], axis=1)


def cylinder_phi(xp):
    """Phi: physical (x, y, z) -> reference (sqrt(x^2 + y^2) + w(z), arccos(x / sqrt(x^2 + y^2)), z)."""
    rho = np.hypot(xp[:, 0], xp[:, 1])
    w, _, _ = cylinder_warp(xp[:, 2])
    return np.stack([rho + w, np.arccos(xp[:, 0] / rho), xp[:, 2]], axis=1)


def cylinder_tensor(xyz, lib=np):
    """The coefficient of the blending example: (1 + z) K (n, 3, 3)."""
    return (1 + xyz[:, 2])[:, None, None] * cylinder_mapping_K(xyz, lib)


def cylinder_tensor_fields_torch(xyz, torch, device="cuda", chunk=1 << 22):
    """tensor_fields(cylinder_tensor(xyz)) with torch on `device` in chunks
    (FP64); returns a (6, n) device tensor."""
    x = torch.as_tensor(xyz, dtype=torch.float64, device=device)
    n = x.shape[0]
    out = torch.empty((6, n), dtype=torch.float64, device=device)
    for c0 in range(0, n, chunk):
        K = cylinder_tensor(x[c0:c0 + chunk], torch)
        for i in range(3):
            out[i, c0:c0 + chunk] = K[:, i, i] - sum(K[:, i, j] for j in range(3) if j != i)
        out[3, c0:c0 + chunk] = K[:, 0, 1]
        out[4, c0:c0 + chunk] = K[:, 0, 2]
        out[5, c0:c0 + chunk] = K[:, 1, 2]
    return out


def _cylinder_factors(xyz):
    """u = A(x) B(y) C(z) with A = sin(pi (x - r1) / (r2 - r1)),
    B = sin(4 y), C = sin(pi z / z1) exp(z / 2), and their first two derivatives."""
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    c = np.pi / (CYL_R2 - CYL_R1)
    A, A1 = np.sin(c * (x - CYL_R1)), c * np.cos(c * (x - CYL_R1))
    A2 = -c * c * A
    B, B1 = np.sin(4 * y), 4 * np.cos(4 * y)
    B2 = -16 * B
    k, e = np.pi / CYL_Z1, np.exp(z / 2)
    C = np.sin(k * z) * e
    C1 = k * np.cos(k * z) * e + C / 2
    C2 = -k * k * C + C1 - C / 4
    return A, A1, A2, B, B1, B2, C, C1, C2


def cylinder_u(xyz):
    """Manufactured solution on the reference box, zero on its boundary:
    sin(pi (x - r1) / (r2 - r1)) sin(4 y) sin(pi z / z1) exp(z / 2)."""
    A, _, _, B, _, _, C, _, _ = _cylinder_factors(xyz)
    return A * B * C


def cylinder_f(xyz):
    """f = -div((1 + z) K grad u) for cylinder_u, written out: with a = 1 + z,
    r = x - w(z), p = w'(z), q = w''(z) and the flux F = a K grad u,
    F_x = a r ((p^2 + 1) u_x + p u_z), F_y = (a / r) u_y, F_z = a r (p u_x + u_z)."""
    A, A1, A2, B, B1, B2, C, C1, C2 = _cylinder_factors(xyz)
    ux, uxx, uyy = A1 * B * C, A2 * B * C, A * B2 * C
    uz, uzz, uxz = A * B * C1, A * B * C2, A1 * B * C1
    x, z = xyz[:, 0], xyz[:, 2]
    w, p, q = cylinder_warp(z)
    r, a = x - w, 1 + z
    dFx = a * ((p * p + 1) * ux + p * uz) + a * r * ((p * p + 1) * uxx + p * uxz)
    dFy = a / r * uyy
    dFz = (r - a * p) * (p * ux + uz) + a * r * (q * ux + p * uxz + uzz)
    return -(dFx + dFy + dFz)


def kuhn_box_mass_rhs(xyz, level, f, nblocks, lo, hi):
    """b = M I_h f for kuhn_box(nblocks, lo, hi) at `level` (the Freudenthal
    triangulation of the grid of nblocks * 2^level cells per axis) at the
    nodes xyz (any order): f sampled on the grid, then the consistent mass
    stencil, one cell volume per cube.  Boundary nodes get the same formula
    (callers zero Dirichlet rows)."""
    lo, hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    N = np.asarray(nblocks) * 2 ** level
    h = (hi - lo) / N
    g = [lo[d] + h[d] * np.arange(N[d] + 1) for d in range(3)]
    X, Y, Z = np.meshgrid(*g, indexing="ij")
    F = f(np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)).reshape(X.shape)
    Fp = np.pad(F, 1)
    B = np.zeros_like(F)
    for (a, b, c), wt in _freudenthal_mass_stencil().items():
        B += wt * Fp[1 + a:N[0] + 2 + a, 1 + b:N[1] + 2 + b, 1 + c:N[2] + 2 + c]
    idx = np.rint((np.asarray(xyz) - lo) / h).astype(np.int64)
    return B[idx[:, 0], idx[:, 1], idx[:, 2]] * float(np.prod(h))
