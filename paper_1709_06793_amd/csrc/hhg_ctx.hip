// hhg_ctx.hip -- host side of the library: macro-mesh topology, per-level
// tables (reference stencils, element matrices, inter-tet node lists, the
// Sec. 4.1 modification), coefficient set-up, and the C ABI of include/hhg.h
// including the multigrid drivers.  All numerical work on vectors runs in the
// kernels of hhg_kernels.hip (and hhg_learned.hip); the host only sets up
// tables and sequences launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/hhg.h"
#include "hhg_internal.h"
#include "hhg_lattice.h"
#include "hhg_learned.h"

using namespace hhg;

namespace {

// ---------------------------------------------------------------- small linear algebra
struct Mat3 {
    double a[3][3];
};

double det3(const Mat3 &m)
{
    return m.a[0][0] * (m.a[1][1] * m.a[2][2] - m.a[1][2] * m.a[2][1]) -
           m.a[0][1] * (m.a[1][0] * m.a[2][2] - m.a[1][2] * m.a[2][0]) +
           m.a[0][2] * (m.a[1][0] * m.a[2][1] - m.a[1][1] * m.a[2][0]);
}

// 4x4 element matrix int_t grad phi_a . grad phi_b of the tet with vertices p[4]
bool element_matrix(const double p[4][3], double E[4][4])
{
    Mat3 J;  // columns p1-p0, p2-p0, p3-p0
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) J.a[r][c] = p[c + 1][r] - p[0][r];
    const double det = det3(J);
    if (!(std::fabs(det) > 0.0)) return false;
    // rows of J^{-1} = gradients of barycentric coordinates 1..3 (cofactors)
    double G[4][3];
    const auto &a = J.a;
    double inv[3][3] = {
        {a[1][1] * a[2][2] - a[1][2] * a[2][1], a[0][2] * a[2][1] - a[0][1] * a[2][2],
         a[0][1] * a[1][2] - a[0][2] * a[1][1]},
        {a[1][2] * a[2][0] - a[1][0] * a[2][2], a[0][0] * a[2][2] - a[0][2] * a[2][0],
         a[0][2] * a[1][0] - a[0][0] * a[1][2]},
        {a[1][0] * a[2][1] - a[1][1] * a[2][0], a[0][1] * a[2][0] - a[0][0] * a[2][1],
         a[0][0] * a[1][1] - a[0][1] * a[1][0]}};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) G[r + 1][c] = inv[r][c] / det;
    for (int c = 0; c < 3; ++c) G[0][c] = -(G[1][c] + G[2][c] + G[3][c]);
    const double vol = std::fabs(det) / 6.0;
    for (int x = 0; x < 4; ++x)
        for (int y = 0; y < 4; ++y)
            E[x][y] = vol * (G[x][0] * G[y][0] + G[x][1] * G[y][1] + G[x][2] * G[y][2]);
    return true;
}

// eigenvalues of a symmetric 3x3 matrix (cyclic Jacobi rotations)
void sym3_eigs(double A[3][3], double ev[3])
{
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        if (off < 1e-300) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {  // A <- A G (columns p,q)
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {  // A <- G^T A (rows p,q)
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
            }
    }
    for (int i = 0; i < 3; ++i) ev[i] = A[i][i];
}

// smallest non-zero eigenvalue of E x = lambda (4I - 11^T) x: on the complement
// of the constants (orthonormal basis B) the right-hand form is 4I
double lambda_min_element(const double E[4][4])
{
    const double r2 = std::sqrt(2.0), r6 = std::sqrt(6.0), r12 = std::sqrt(12.0);
    const double B[4][3] = {{1 / r2, 1 / r6, 1 / r12},
                            {-1 / r2, 1 / r6, 1 / r12},
                            {0, -2 / r6, 1 / r12},
                            {0, 0, -3 / r12}};
    double R[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) s += B[a][i] * E[a][b] * B[b][j];
            R[i][j] = s;
        }
    double ev[3];
    sym3_eigs(R, ev);
    return std::min(ev[0], std::min(ev[1], ev[2])) / 4.0;
}

// dense inverse with partial pivoting (Gauss-Jordan), in place; false if singular
bool invert_dense(std::vector<double> &A, int n)
{
    std::vector<double> I((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)p * n + c])) p = r;
        if (!(std::fabs(A[(size_t)p * n + c]) > 0.0)) return false;
        if (p != c)
            for (int k = 0; k < n; ++k) {
                std::swap(A[(size_t)p * n + k], A[(size_t)c * n + k]);
                std::swap(I[(size_t)p * n + k], I[(size_t)c * n + k]);
            }
        const double piv = A[(size_t)c * n + c];
        for (int k = 0; k < n; ++k) {
            A[(size_t)c * n + k] /= piv;
            I[(size_t)c * n + k] /= piv;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = A[(size_t)r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
                I[(size_t)r * n + k] -= f * I[(size_t)c * n + k];
            }
        }
    }
    A.swap(I);
    return true;
}

int popcount4(int z) { return (z & 1) + ((z >> 1) & 1) + ((z >> 2) & 1) + ((z >> 3) & 1); }

// ---------------------------------------------------------------- topology
// Geometric conformity of a macro mesh whose tets already have positive
// volume and whose faces are each held by at most two tets.  Shared
// primitives are recognised by vertex ids, so a mesh is non-conforming when
// geometry meets without ids agreeing:
//   * two vertex ids at the same point;
//   * a vertex on an edge or a face of a tet that does not hold it (a hanging
//     node: the finer side's lattice would not match the coarser side's);
//   * two faces held by one tet each that lie in one plane and overlap (the
//     two sides of a quadrilateral split along different diagonals).
// Candidates are found by sorting vertices and faces by their x extent.
// Returns an empty string for a conforming mesh, else what was found.
static std::string conformity_error(const std::vector<double> &X, const std::vector<int> &tet, int nv, int nt,
                                    const std::vector<std::array<int, 2>> &edges,
                                    const std::vector<std::array<int, 3>> &faces, const std::vector<int> &f_val)
{
    auto P = [&](int v, int a) { return X[3 * v + a]; };
    std::vector<int> used;
    {
        std::vector<uint8_t> u(nv, 0);
        for (int i = 0; i < 4 * nt; ++i) u[tet[i]] = 1;
        for (int v = 0; v < nv; ++v)
            if (u[v]) used.push_back(v);
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int v : used)
        for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], P(v, a)); hi[a] = std::max(hi[a], P(v, a)); }
    double diam = 0.0;
    for (int a = 0; a < 3; ++a) diam = std::max(diam, hi[a] - lo[a]);
    const double eps = 1e-10 * diam;
    std::vector<int> byx = used;
    std::sort(byx.begin(), byx.end(), [&](int a, int b) { return P(a, 0) < P(b, 0); });
    auto in_range = [&](double x0, double x1, auto fn) {
        auto it = std::lower_bound(byx.begin(), byx.end(), x0 - eps, [&](int v, double x) { return P(v, 0) < x; });
        for (; it != byx.end() && P(*it, 0) <= x1 + eps; ++it)
            if (fn(*it)) return true;
        return false;
    };
    char buf[160];
    // coincident vertices
    for (size_t q = 0; q + 1 < byx.size(); ++q) {
        const int a = byx[q];
        bool hit = in_range(P(a, 0), P(a, 0), [&](int b) {
            if (b == a) return false;
            double d = 0.0;
            for (int c = 0; c < 3; ++c) d = std::max(d, std::fabs(P(a, c) - P(b, c)));
            if (d <= eps) {
                snprintf(buf, sizeof buf, "vertices %d and %d coincide", std::min(a, b), std::max(a, b));
                return true;
            }
            return false;
        });
        if (hit) return buf;
    }
    // a vertex inside an edge
    for (const auto &e : edges) {
        const int a = e[0], b = e[1];
        double d[3], len2 = 0.0;
        for (int c = 0; c < 3; ++c) { d[c] = P(b, c) - P(a, c); len2 += d[c] * d[c]; }
        bool hit = in_range(std::min(P(a, 0), P(b, 0)), std::max(P(a, 0), P(b, 0)), [&](int v) {
            if (v == a || v == b) return false;
            double t = 0.0;
            for (int c = 0; c < 3; ++c) t += (P(v, c) - P(a, c)) * d[c];
            t /= len2;
            if (t <= 0.0 || t >= 1.0) return false;
            double dist = 0.0;
            for (int c = 0; c < 3; ++c) dist = std::max(dist, std::fabs(P(a, c) + t * d[c] - P(v, c)));
            if (dist <= eps) {
                snprintf(buf, sizeof buf, "vertex %d lies on macro edge (%d,%d)", v, a, b);
                return true;
            }
            return false;
        });
        if (hit) return buf;
    }
    // barycentric coordinates of point x in the plane of face f (false if
    // the point is off the plane)
    auto face_bary = [&](const std::array<int, 3> &f, const double *x, double w[3]) {
        double e1[3], e2[3], r[3], nrm[3];
        for (int c = 0; c < 3; ++c) {
            e1[c] = P(f[1], c) - P(f[0], c);
            e2[c] = P(f[2], c) - P(f[0], c);
            r[c] = x[c] - P(f[0], c);
        }
        nrm[0] = e1[1] * e2[2] - e1[2] * e2[1];
        nrm[1] = e1[2] * e2[0] - e1[0] * e2[2];
        nrm[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double n2 = nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2];
        const double off = (r[0] * nrm[0] + r[1] * nrm[1] + r[2] * nrm[2]) / std::sqrt(n2);
        if (std::fabs(off) > eps) return false;
        const double d11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
        const double d12 = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
        const double d22 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
        const double r1 = r[0] * e1[0] + r[1] * e1[1] + r[2] * e1[2];
        const double r2 = r[0] * e2[0] + r[1] * e2[1] + r[2] * e2[2];
        const double det = d11 * d22 - d12 * d12;
        w[1] = (d22 * r1 - d12 * r2) / det;
        w[2] = (d11 * r2 - d12 * r1) / det;
        w[0] = 1.0 - w[1] - w[2];
        return true;
    };
    const double beps = 1e-10;
    // a vertex inside a face (edges are covered above)
    for (const auto &f : faces) {
        const double x0 = std::min({P(f[0], 0), P(f[1], 0), P(f[2], 0)});
        const double x1 = std::max({P(f[0], 0), P(f[1], 0), P(f[2], 0)});
        bool hit = in_range(x0, x1, [&](int v) {
            if (v == f[0] || v == f[1] || v == f[2]) return false;
            double x[3] = {P(v, 0), P(v, 1), P(v, 2)}, w[3];
            if (!face_bary(f, x, w)) return false;
            if (w[0] > beps && w[1] > beps && w[2] > beps) {
                snprintf(buf, sizeof buf, "vertex %d lies on macro face (%d,%d,%d)", v, f[0], f[1], f[2]);
                return true;
            }
            return false;
        });
        if (hit) return buf;
    }
    // coplanar overlapping faces held by one tet each: some point strictly
    // inside one triangle (its centroid or a point just inside an edge
    // midpoint or a corner) lies strictly inside the other
    std::vector<int> bf;
    for (size_t f = 0; f < faces.size(); ++f)
        if (f_val[f] == 1) bf.push_back((int)f);
    std::vector<std::array<double, 2>> fx(faces.size());
    for (int f : bf) {
        const auto &F = faces[f];
        fx[f] = {std::min({P(F[0], 0), P(F[1], 0), P(F[2], 0)}), std::max({P(F[0], 0), P(F[1], 0), P(F[2], 0)})};
    }
    std::sort(bf.begin(), bf.end(), [&](int a, int b) { return fx[a][0] < fx[b][0]; });
    for (size_t qa = 0; qa < bf.size(); ++qa) {
        const auto &A = faces[bf[qa]];
        for (size_t qb = qa + 1; qb < bf.size() && fx[bf[qb]][0] <= fx[bf[qa]][1] + eps; ++qb) {
            const auto &B = faces[bf[qb]];
            for (int pass = 0; pass < 2; ++pass) {
                const auto &S = pass ? B : A, &D = pass ? A : B;
                // sample points strictly inside S
                const double wts[7][3] = {{1 / 3., 1 / 3., 1 / 3.}, {0.98, 0.01, 0.01}, {0.01, 0.98, 0.01},
                                          {0.01, 0.01, 0.98},       {0.495, 0.495, 0.01}, {0.01, 0.495, 0.495},
                                          {0.495, 0.01, 0.495}};
                for (const auto &wt : wts) {
                    double x[3], w[3];
                    for (int c = 0; c < 3; ++c) x[c] = wt[0] * P(S[0], c) + wt[1] * P(S[1], c) + wt[2] * P(S[2], c);
                    if (face_bary(D, x, w) && w[0] > beps && w[1] > beps && w[2] > beps) {
                        snprintf(buf, sizeof buf, "macro faces (%d,%d,%d) and (%d,%d,%d) overlap", A[0], A[1], A[2],
                                 B[0], B[1], B[2]);
                        return buf;
                    }
                }
            }
        }
    }
    return std::string();
}

struct Topology {
    int nv = 0, nt = 0;
    std::vector<double> X;
    std::vector<int> tet;
    std::vector<int> vpos;                      // vertex id -> canonical index, -1 unused
    int nvu = 0;
    std::vector<std::array<int, 2>> edges;      // sorted
    std::vector<std::array<int, 3>> faces;      // sorted
    std::vector<int> v_val, e_val, f_val;       // number of tets holding the primitive
    std::vector<uint8_t> v_bnd, e_bnd, f_bnd;

    int find_edge(int a, int b) const
    {
        std::array<int, 2> key = {std::min(a, b), std::max(a, b)};
        auto it = std::lower_bound(edges.begin(), edges.end(), key);
        return (it != edges.end() && *it == key) ? (int)(it - edges.begin()) : -1;
    }
    int find_face(int a, int b, int c) const
    {
        std::array<int, 3> key = {a, b, c};
        std::sort(key.begin(), key.end());
        auto it = std::lower_bound(faces.begin(), faces.end(), key);
        return (it != faces.end() && *it == key) ? (int)(it - faces.begin()) : -1;
    }
    // global primitive of tet t's local primitive with zero pattern zp:
    // returns dimension (0 vertex .. 3 tet) and its index
    void primitive(int t, int zp, int &dim, int &idx, std::vector<int> *verts = nullptr) const
    {
        int v[4], c = 0;
        for (int a = 0; a < 4; ++a)
            if (!((zp >> a) & 1)) v[c++] = tet[4 * t + a];
        dim = c - 1;
        if (verts) verts->assign(v, v + c);
        if (c == 4) idx = t;
        else if (c == 3) idx = find_face(v[0], v[1], v[2]);
        else if (c == 2) idx = find_edge(v[0], v[1]);
        else idx = v[0];
    }
    int valence(int t, int zp) const
    {
        int dim, idx;
        primitive(t, zp, dim, idx);
        return dim == 3 ? 1 : dim == 2 ? f_val[idx] : dim == 1 ? e_val[idx] : v_val[idx];
    }
    bool dirichlet(int t, int zp) const
    {
        int dim, idx;
        primitive(t, zp, dim, idx);
        return dim == 3 ? false : dim == 2 ? f_bnd[idx] : dim == 1 ? e_bnd[idx] : v_bnd[idx];
    }
};

// ---------------------------------------------------------------- per-level data
template <typename T>
struct DBuf {
    T *p = nullptr;
    int64_t n = 0;
};

struct Level {
    int l = 0, n = 0, S = 0, bpt = 0;
    int64_t Spad = 0, n_slots = 0, n_nodes = 0, n_unknowns = 0;
    // per-tet tables
    std::vector<double> h_sten, h_emat, h_rstw;
    std::vector<uint16_t> h_dmask, h_smask;
    double *sten64 = nullptr, *emat64 = nullptr, *rstw64 = nullptr;
    float *sten32 = nullptr, *emat32 = nullptr, *rstw32 = nullptr;
    uint16_t *dmask = nullptr, *smask = nullptr;
    // column-marching work items and boundary slot list (same for every tet)
    std::vector<uint32_t> h_items;  // pairs (t0, k0 | k1 << 16)
    std::vector<uint32_t> h_bnd;
    uint2 *items = nullptr;
    std::vector<uint32_t> h_itemsL;  // block items of the LDS-staged kernel
    uint2 *itemsL = nullptr;
    int n_itemsL = 0, kcL = 0;
    std::vector<uint32_t> h_items2, h_items2f;  // two-rows-per-lane kernel (FP64, FP32)
    uint2 *items2 = nullptr, *items2f = nullptr;
    int n_items2 = 0, kc2 = 0, n_items2f = 0, kc2f = 0;
    uint32_t *bnd = nullptr;
    int n_items = 0, n_bnd = 0, kc = 0;
    // shared nodes
    int n_shared = 0;
    std::vector<int32_t> h_sh_off;
    std::vector<uint64_t> h_sh_copy;
    int32_t *sh_off = nullptr;
    uint64_t *sh_copy = nullptr;
    int sh_w = 0;
    int64_t *sh_nb = nullptr, *sh_self = nullptr, *sh_cslot = nullptr;
    uint32_t *sh_nb32 = nullptr, *sh_self32 = nullptr, *sh_cslot32 = nullptr, *sh_nbs32 = nullptr;
    int8_t *sh_map = nullptr;  // [copy][16]: entry of direction d, -1 if none
    // the scaled operator's own (narrower) pattern
    int sh_ws = 0;
    int64_t *sh_nbs = nullptr;
    int8_t *sh_maps = nullptr;
    double *sh_css64 = nullptr;
    float *sh_css32 = nullptr;
    // the same for the tensor operator's (wider) pattern
    int sh_wt = 0;
    int64_t *sh_nbt = nullptr;
    int8_t *sh_mapt = nullptr;
    std::vector<uint8_t> h_sh_prim;  // macro primitive of each shared node (1 vertex, 2 edge, 4 face)
    uint8_t *sh_prim = nullptr;
    double *sh_cs64 = nullptr, *sh_cn64 = nullptr, *sh_ct64 = nullptr, *sh_ctn64 = nullptr;
    float *sh_cs32 = nullptr, *sh_cn32 = nullptr, *sh_ct32 = nullptr, *sh_ctn32 = nullptr;
    // coefficient dependent
    // tensor operator: per-tet component stencils and the six coefficient fields
    std::vector<double> h_tsten, h_temat;
    double *tsten64 = nullptr, *kt64 = nullptr, *kp64 = nullptr, *temat64 = nullptr;
    float *tsten32 = nullptr, *kt32 = nullptr, *kp32 = nullptr, *temat32 = nullptr;
    double *k64 = nullptr, *invd64 = nullptr;
    float *k32 = nullptr, *invd32 = nullptr;
    double lam = 0.0;
    // the other operators a cycle can run on (index op - 1, op as
    // hhg_ctx_s::op): inverse diagonal and Gershgorin bound
    double *oinvd64[4] = {nullptr, nullptr, nullptr, nullptr};
    float *oinvd32[4] = {nullptr, nullptr, nullptr, nullptr};
    double olam[4] = {0.0, 0.0, 0.0, 0.0};
    // work vectors
    double *r64 = nullptr, *d64 = nullptr, *f64 = nullptr, *u64 = nullptr;
    float *r32 = nullptr, *d32 = nullptr, *f32 = nullptr, *u32 = nullptr;
    // modification corrections
    int n_corr_rows = 0;
    int64_t n_corr = 0;
    int32_t *c_off = nullptr, *p_off = nullptr;
    int64_t *c_self = nullptr, *c_nb = nullptr, *p_slot = nullptr;
    double *c_d64 = nullptr, *c_base = nullptr;
    float *c_d32 = nullptr;
    uint8_t *c_nbdir = nullptr;
    uint8_t *c_prim = nullptr;
    // stored stencils (allocated by hhg_store_stencils, refreshed with k)
    double *st64 = nullptr;
    float *st32 = nullptr;
    // learned correction: log k (FP32), ownership mask and FP32 scratch
    float *logk32 = nullptr;
    uint8_t *own = nullptr;
    float *lt[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    int64_t partial_bound = 0;  // block partials any reduction at this level writes
    // geometric coarse coefficients (this level as the coarse one): the nodes
    // on macro primitives with their distinct fine support nodes and weights
    // (CSR) and their copies (CSR)
    bool cg_ready = false;
    int cg_n = 0;
    int32_t *cg_off = nullptr, *cg_coff = nullptr;
    int64_t *cg_fslot = nullptr, *cg_cslot = nullptr;
    double *cg_w = nullptr;
    double *ubak = nullptr;  // last accepted iterate of a learned solve
    double *uprobe = nullptr;  // a learned solve's plain-cycle probe result
    // canonical maps (built on first use); slot2canon holds -(c+1) for a
    // Dirichlet slot of node c
    int32_t *slot2canon = nullptr;
    int64_t *canon2slot = nullptr;
    std::vector<int64_t> h_poff;  // interior nodes in planes 1..k-1
};

}  // namespace

struct CoarseInv {
    int cu = 0;
    double *ainv = nullptr;
    int64_t *cgather = nullptr;
    int32_t *ccoff = nullptr;
    int64_t *ccslot = nullptr;
    double *cf = nullptr;  // the gathered right-hand side (cu values)
};

struct hhg_ctx_s {
    Topology topo;
    // the device's copy of the allocation-free entry point's static scratch
    // array (resolved at creation, with the device current)
    double *noalloc_scratch = nullptr;
    int max_level = 0, coarse = 0;
    uint32_t flags = 0;
    hipStream_t stream = nullptr;
    std::vector<Level> lv;
    bool have_k = false;
    bool have_tk = false;  // tensor coefficient set
    std::vector<void *> allocs;
    double *partial = nullptr;
    int64_t partial_cap = 0;
    double *dscalar = nullptr;  // device scalars
    double *hscalar = nullptr;  // pinned host scalars
    int *dflag = nullptr;
    // the operator residuals, smoothers and coarse solves run on: 0 scalar
    // scaled (with the modification), 1 tensor scaled, 2 tensor nodal, 3
    // scalar nodal, 4 primitive-mixed with nodal rows on mix_mask
    int op = 0;
    int mix_mask = 0;
    CoarseInv co[5];  // dense coarse inverses per operator
    // solver state of operators 1..4 (index op - 1): built, for which coarse
    // level, and for the mixed operator which primitive mask
    bool oready[4] = {false, false, false, false};
    int oco_level[4] = {-1, -1, -1, -1};
    int omask = 0;
    std::string err;
    // learned correction
    LearnedState learned;
    // V-cycles of the solve loops replayed as captured HIP graphs (one per
    // level, cycle shape, operator, precision and vector pair; entries of an
    // older epoch are stale: the epoch moves whenever state a cycle's kernels
    // read by value or pointer is rebuilt).  Off by default: replays measured
    // 4-15% slower than stream launches for 10 V-cycles at 6-tet levels 4-8.
    bool graphs = false;
    uint64_t graph_epoch = 0;
    hipStream_t gstream = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};
    struct GraphKey {
        int level, pre, post, sm, op, mask, dt, variant;
        const void *f;
        const void *u;
        uint64_t epoch;
        bool operator<(const GraphKey &o) const
        {
            return std::tie(level, pre, post, sm, op, mask, dt, variant, f, u, epoch) <
                   std::tie(o.level, o.pre, o.post, o.sm, o.op, o.mask, o.dt, o.variant, o.f, o.u, o.epoch);
        }
    };
    std::map<GraphKey, std::pair<hipGraph_t, hipGraphExec_t>> gcache;
    // optional timing of the operator kernels of hhg_apply_scaled (event pairs)
    bool timing = false;
    std::vector<hipEvent_t> tev;  // start/end pairs
    size_t tev_used = 0;          // pairs recorded
};

// Scratch of hhg_residual_noalloc: the residual norm's per-block partials
// (from element NOALLOC_PARTIAL_AT on) and the reduced value (element 0).
// Each GPU holds its own copy from the library's load until the process
// ends.  Host code must not use the array's name as a device address: the
// device address comes from hipGetSymbolAddress, once per device.
constexpr int64_t NOALLOC_SCRATCH_DOUBLES = int64_t(1) << 20;  // 8 MiB
constexpr int64_t NOALLOC_PARTIAL_AT = 32;                      // 256-byte aligned
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
double *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// the current device's address of `scratch` (looked up on the first call
// for that device, then kept); nullptr with *err set on failure
double *noalloc_scratch_address(hipError_t *err)
{
    int dev = -1;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (*err != hipSuccess || !p) return nullptr;
        g_noalloc_ptr[dev] = static_cast<double *>(p);
    }
    *err = hipSuccess;
    return g_noalloc_ptr[dev];
}

}  // namespace

namespace {

thread_local std::string g_create_error;

hhg_status fail(hhg_ctx c, hhg_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_create_error = buf;
    return code;
}

#define HIPCHK(ctx, ...)                                                                    \
    do {                                                                                    \
        hipError_t e_ = (__VA_ARGS__);                                                      \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), HHG_EHIP, "%s failed: %s", #__VA_ARGS__,                     \
                        hipGetErrorString(e_));                                             \
    } while (0)

// free memory that dalloc/upload gave out
void dfree(hhg_ctx c, void *p)
{
    if (!p) return;
    auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
    if (it != c->allocs.end()) c->allocs.erase(it);
    (void)hipFree(p);
}

template <typename T>
hhg_status dalloc(hhg_ctx c, T **p, int64_t n)
{
    *p = nullptr;
    if (n <= 0) n = 1;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, (size_t)n * sizeof(T));
    if (e != hipSuccess) return fail(c, HHG_ENOMEM, "hipMalloc of %lld bytes failed: %s",
                                     (long long)(n * sizeof(T)), hipGetErrorString(e));
    c->allocs.push_back(q);
    *p = (T *)q;
    return HHG_OK;
}

template <typename T>
hhg_status upload(hhg_ctx c, T **p, const std::vector<T> &h)
{
    hhg_status s = dalloc(c, p, (int64_t)h.size());
    if (s) return s;
    if (!h.empty()) HIPCHK(c, hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return HHG_OK;
}

hipStream_t pick(hhg_ctx c, void *s) { return s ? (hipStream_t)s : c->stream; }

#define TRY(expr)                      \
    do {                               \
        hhg_status s_ = (expr);        \
        if (s_ < 0) return s_;         \
    } while (0)

// element-shape pairs (t, a, b) whose edge a->b runs along direction d
struct EdgeUse {
    int t, a, b;
};
std::vector<EdgeUse> g_edge_use[NDIR];
void init_edge_use()
{
    if (!g_edge_use[0].empty()) return;
    for (int t = 0; t < NTYPE; ++t)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                if (a == b) continue;
                const int d = dir_index(TYPE_OFF[t][b][0] - TYPE_OFF[t][a][0],
                                        TYPE_OFF[t][b][1] - TYPE_OFF[t][a][1],
                                        TYPE_OFF[t][b][2] - TYPE_OFF[t][a][2]);
                g_edge_use[d].push_back({t, a, b});
            }
}

// physical coordinates of lattice point (i,j,k) of tet t at n intervals
void lattice_point(const Topology &tp, int t, int n, double i, double j, double k, double x[3])
{
    const double *v0 = &tp.X[3 * tp.tet[4 * t]], *v1 = &tp.X[3 * tp.tet[4 * t + 1]],
                 *v2 = &tp.X[3 * tp.tet[4 * t + 2]], *v3 = &tp.X[3 * tp.tet[4 * t + 3]];
    for (int c = 0; c < 3; ++c)
        x[c] = v0[c] + (i * (v1[c] - v0[c]) + j * (v2[c] - v0[c]) + k * (v3[c] - v0[c])) / n;
}

// the six element matrices of tet t at n intervals
// element matrix of one tensor component D = c.grad: |t| (c.g_a)(c.g_b)
bool element_matrix_dir(const double p[4][3], const double cdir[3], double E[4][4])
{
    double L[4][4];
    if (!element_matrix(p, L)) return false;  // validity (non-zero volume)
    Mat3 J;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) J.a[r][c] = p[c + 1][r] - p[0][r];
    const double det = det3(J);
    const auto &a = J.a;
    const double inv[3][3] = {
        {a[1][1] * a[2][2] - a[1][2] * a[2][1], a[0][2] * a[2][1] - a[0][1] * a[2][2],
         a[0][1] * a[1][2] - a[0][2] * a[1][1]},
        {a[1][2] * a[2][0] - a[1][0] * a[2][2], a[0][0] * a[2][2] - a[0][2] * a[2][0],
         a[0][2] * a[1][0] - a[0][0] * a[1][2]},
        {a[1][0] * a[2][1] - a[1][1] * a[2][0], a[0][1] * a[2][0] - a[0][0] * a[2][1],
         a[0][0] * a[1][1] - a[0][1] * a[1][0]}};
    double dg[4] = {0, 0, 0, 0};
    for (int r = 0; r < 3; ++r) {
        dg[r + 1] = (inv[r][0] * cdir[0] + inv[r][1] * cdir[1] + inv[r][2] * cdir[2]) / det;
        dg[0] -= dg[r + 1];
    }
    const double vol = std::fabs(det) / 6.0;
    for (int x = 0; x < 4; ++x)
        for (int y = 0; y < 4; ++y) E[x][y] = vol * dg[x] * dg[y];
    return true;
}

bool type_matrices(const Topology &tp, int t, int n, double E[NTYPE][4][4])
{
    for (int ty = 0; ty < NTYPE; ++ty) {
        double p[4][3];
        for (int a = 0; a < 4; ++a)
            lattice_point(tp, t, n, TYPE_OFF[ty][a][0], TYPE_OFF[ty][a][1], TYPE_OFF[ty][a][2], p[a]);
        if (!element_matrix(p, E[ty])) return false;
    }
    return true;
}

// representative lattice point (with nrep = 8 intervals) of the primitive with
// zero pattern zp: every non-zero barycentric weight is at least 2
void representative(int zp, int &i, int &j, int &k)
{
    int w[4] = {0, 0, 0, 0}, idx[4], c = 0;
    for (int a = 0; a < 4; ++a)
        if (!((zp >> a) & 1)) idx[c++] = a;
    for (int q = 0; q < 8; ++q) w[idx[q % c]] += 1;
    i = w[1]; j = w[2]; k = w[3];
}

bool element_valid(int n, int bi, int bj, int bk, int t)
{
    for (int v = 0; v < 4; ++v)
        if (!in_lattice(n, bi + TYPE_OFF[t][v][0], bj + TYPE_OFF[t][v][1], bk + TYPE_OFF[t][v][2]))
            return false;
    return true;
}

// canonical index of lattice point (i,j,k) of tet t at n intervals; poff[k] =
// number of tet-interior nodes in planes 1..k-1
int64_t canon_index(const Topology &tp, int t, int n, int i, int j, int k, const int64_t *poff)
{
    const int w[4] = {n - i - j - k, i, j, k};
    int vid[4], ww[4], c = 0;
    for (int a = 0; a < 4; ++a)
        if (w[a] > 0) { vid[c] = tp.tet[4 * t + a]; ww[c] = w[a]; ++c; }
    const int64_t N = n, EN = N - 1, FN = (N - 1) * (N - 2) / 2, TN = (N - 1) * (N - 2) * (N - 3) / 6;
    const int64_t off_e = tp.nvu, off_f = off_e + (int64_t)tp.edges.size() * EN,
                  off_t = off_f + (int64_t)tp.faces.size() * FN;
    if (c == 4) {
        // interior: k outer, then j, then i; row jj of plane k holds M - jj
        // points, M = n-1-k
        const int64_t M = N - 1 - k;
        const int64_t loc = poff[k] + (int64_t)(j - 1) * M - (int64_t)(j - 1) * j / 2;
        return off_t + (int64_t)t * TN + loc + (i - 1);
    }
    for (int a = 1; a < c; ++a)  // sort by vertex id
        for (int b = a; b > 0 && vid[b - 1] > vid[b]; --b) {
            std::swap(vid[b - 1], vid[b]);
            std::swap(ww[b - 1], ww[b]);
        }
    if (c == 1) return tp.vpos[vid[0]];
    if (c == 2) return off_e + (int64_t)tp.find_edge(vid[0], vid[1]) * EN + (ww[1] - 1);
    const int64_t s = ww[1], tt = ww[2];
    return off_f + (int64_t)tp.find_face(vid[0], vid[1], vid[2]) * FN + (tt - 1) * (N - 1) -
           (tt - 1) * tt / 2 + (s - 1);
}

template <typename T>
LevelView<T> view(const hhg_ctx c, int l);

template <>
LevelView<double> view<double>(const hhg_ctx c, int l)
{
    const Level &L = c->lv[l];
    LevelView<double> v;
    v.n = L.n; v.n_tet = c->topo.nt; v.S = L.S; v.Spad = L.Spad; v.bpt = L.bpt;
    v.sten = L.sten64; v.emat = L.emat64; v.rstw = L.rstw64;
    v.dmask = L.dmask; v.smask = L.smask; v.kap = L.k64;
    v.n_shared = L.n_shared; v.sh_off = L.sh_off; v.sh_copy = L.sh_copy;
    v.items = L.items; v.n_items = L.n_items; v.vpt = (L.n_items + 3) / 4;
    v.sh_w = L.sh_w; v.sh_nb = L.sh_nb; v.sh_self = L.sh_self; v.sh_cslot = L.sh_cslot;
    v.sh_cs = L.sh_cs64; v.sh_cn = L.sh_cn64; v.sh_prim = L.sh_prim;
    v.sh_ws = L.sh_ws; v.sh_nbs = L.sh_nbs; v.sh_css = L.sh_css64;
    v.sh_nb32 = L.sh_nb32; v.sh_self32 = L.sh_self32; v.sh_cslot32 = L.sh_cslot32; v.sh_nbs32 = L.sh_nbs32;
    v.sh_wt = L.sh_wt; v.sh_nbt = L.sh_nbt; v.sh_ct = L.sh_ct64; v.sh_ctn = L.sh_ctn64;
    v.tsten = L.tsten64; v.kt = L.kt64; v.kp = L.kp64; v.temat = L.temat64;
    v.items2 = L.items2; v.n_items2 = L.n_items2; v.vpt2 = (L.n_items2 + 3) / 4;
    v.itemsL = L.itemsL; v.n_itemsL = L.n_itemsL;
    v.bnd = L.bnd; v.n_bnd = L.n_bnd; v.bpt2 = (L.n_bnd + BLOCK - 1) / BLOCK;
    return v;
}
template <>
LevelView<float> view<float>(const hhg_ctx c, int l)
{
    const Level &L = c->lv[l];
    LevelView<float> v;
    v.n = L.n; v.n_tet = c->topo.nt; v.S = L.S; v.Spad = L.Spad; v.bpt = L.bpt;
    v.sten = L.sten32; v.emat = L.emat32; v.rstw = L.rstw32;
    v.dmask = L.dmask; v.smask = L.smask; v.kap = L.k32;
    v.n_shared = L.n_shared; v.sh_off = L.sh_off; v.sh_copy = L.sh_copy;
    v.items = L.items; v.n_items = L.n_items; v.vpt = (L.n_items + 3) / 4;
    v.sh_w = L.sh_w; v.sh_nb = L.sh_nb; v.sh_self = L.sh_self; v.sh_cslot = L.sh_cslot;
    v.sh_cs = L.sh_cs32; v.sh_cn = L.sh_cn32; v.sh_prim = L.sh_prim;
    v.sh_ws = L.sh_ws; v.sh_nbs = L.sh_nbs; v.sh_css = L.sh_css32;
    v.sh_nb32 = L.sh_nb32; v.sh_self32 = L.sh_self32; v.sh_cslot32 = L.sh_cslot32; v.sh_nbs32 = L.sh_nbs32;
    v.sh_wt = L.sh_wt; v.sh_nbt = L.sh_nbt; v.sh_ct = L.sh_ct32; v.sh_ctn = L.sh_ctn32;
    v.tsten = L.tsten32; v.kt = L.kt32; v.kp = L.kp32; v.temat = L.temat32;
    v.items2 = L.items2f; v.n_items2 = L.n_items2f; v.vpt2 = (L.n_items2f + 3) / 4;
    v.itemsL = L.itemsL; v.n_itemsL = L.n_itemsL;
    v.bnd = L.bnd; v.n_bnd = L.n_bnd; v.bpt2 = (L.n_bnd + BLOCK - 1) / BLOCK;
    return v;
}

template <typename T>
CorrView<T> corr(const hhg_ctx c, int l);
template <>
CorrView<double> corr<double>(const hhg_ctx c, int l)
{
    const Level &L = c->lv[l];
    return CorrView<double>{L.n_corr_rows, L.c_off, L.c_self, L.c_nb, L.c_d64, L.c_base, L.c_nbdir,
                            L.p_off, L.p_slot, L.c_prim};
}
template <>
CorrView<float> corr<float>(const hhg_ctx c, int l)
{
    const Level &L = c->lv[l];
    return CorrView<float>{L.n_corr_rows, L.c_off, L.c_self, L.c_nb, L.c_d32, L.c_base, L.c_nbdir,
                           L.p_off, L.p_slot, L.c_prim};
}

template <typename T> T *&work_r(Level &L);
template <> double *&work_r<double>(Level &L) { return L.r64; }
template <> float *&work_r<float>(Level &L) { return L.r32; }
template <typename T> T *&work_d(Level &L);
template <> double *&work_d<double>(Level &L) { return L.d64; }
template <> float *&work_d<float>(Level &L) { return L.d32; }
template <typename T> T *&work_f(Level &L);
template <> double *&work_f<double>(Level &L) { return L.f64; }
template <> float *&work_f<float>(Level &L) { return L.f32; }
template <typename T> T *&work_u(Level &L);
template <> double *&work_u<double>(Level &L) { return L.u64; }
template <> float *&work_u<float>(Level &L) { return L.u32; }
template <typename T> T *&invd(Level &L);
template <> double *&invd<double>(Level &L) { return L.invd64; }
template <> float *&invd<float>(Level &L) { return L.invd32; }

// ---------------------------------------------------------------- level set-up
hhg_status build_level(hhg_ctx c, int l)
{
    const Topology &tp = c->topo;
    Level &L = c->lv[l];
    L.l = l;
    L.n = 1 << l;
    L.S = (int)tet_count(L.n);
    L.Spad = ((int64_t)L.S + 63) / 64 * 64;
    L.bpt = (L.S + BLOCK - 1) / BLOCK;
    L.n_slots = (int64_t)tp.nt * L.Spad;
    const int64_t N = L.n;
    L.n_nodes = tp.nvu + (int64_t)tp.edges.size() * (N - 1) + (int64_t)tp.faces.size() * (N - 1) * (N - 2) / 2 +
                (int64_t)tp.nt * (N - 1) * (N - 2) * (N - 3) / 6;
    // unknowns: nodes not on a Dirichlet primitive
    int64_t nu = 0;
    for (int v = 0; v < tp.nv; ++v)
        if (tp.vpos[v] >= 0 && !tp.v_bnd[v]) ++nu;
    for (size_t e = 0; e < tp.edges.size(); ++e)
        if (!tp.e_bnd[e]) nu += N - 1;
    for (size_t f = 0; f < tp.faces.size(); ++f)
        if (!tp.f_bnd[f]) nu += (N - 1) * (N - 2) / 2;
    nu += (int64_t)tp.nt * (N - 1) * (N - 2) * (N - 3) / 6;
    L.n_unknowns = nu;
    L.h_poff.assign(L.n + 2, 0);
    for (int k = 1; k <= L.n; ++k) {
        const int64_t M = N - 1 - k;
        L.h_poff[k + 1] = L.h_poff[k] + (M >= 2 ? (M - 1) * M / 2 : 0);
    }

    // per-tet tables
    L.h_sten.assign((size_t)tp.nt * TET_STENCIL, 0.0);
    L.h_rstw.assign((size_t)tp.nt * TET_STENCIL, 0.0);
    L.h_emat.assign((size_t)tp.nt * TET_EMAT, 0.0);
    L.h_dmask.assign(tp.nt, 0);
    L.h_smask.assign(tp.nt, 0);
    for (int t = 0; t < tp.nt; ++t) {
        double E[NTYPE][4][4];
        if (!type_matrices(tp, t, L.n, E)) return fail(c, HHG_EMESH, "tet %d is degenerate", t);
        for (int ty = 0; ty < NTYPE; ++ty)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    L.h_emat[(size_t)t * TET_EMAT + ty * 16 + a * 4 + b] = E[ty][a][b] / 4.0;
        for (int zp = 0; zp < 15; ++zp) {
            if (popcount4(zp) == 4) continue;
            if (tp.dirichlet(t, zp)) L.h_dmask[t] |= (uint16_t)(1u << zp);
            else if (zp != 0) L.h_smask[t] |= (uint16_t)(1u << zp);
            int ri, rj, rk;
            representative(zp, ri, rj, rk);
            double st[NDIR + 1] = {0};
            int cnt[NDIR] = {0};
            for (int ty = 0; ty < NTYPE; ++ty)
                for (int a = 0; a < 4; ++a) {
                    const int bi = ri - TYPE_OFF[ty][a][0], bj = rj - TYPE_OFF[ty][a][1],
                              bk = rk - TYPE_OFF[ty][a][2];
                    if (!element_valid(8, bi, bj, bk, ty)) continue;
                    for (int b = 0; b < 4; ++b) {
                        const int d = dir_index(TYPE_OFF[ty][b][0] - TYPE_OFF[ty][a][0],
                                                TYPE_OFF[ty][b][1] - TYPE_OFF[ty][a][1],
                                                TYPE_OFF[ty][b][2] - TYPE_OFF[ty][a][2]);
                        st[d] += E[ty][a][b];
                        if (d < NDIR) cnt[d]++;
                    }
                }
            double *row = &L.h_sten[(size_t)t * TET_STENCIL + zp * KIND_STRIDE];
            double *rw = &L.h_rstw[(size_t)t * TET_STENCIL + zp * KIND_STRIDE];
            for (int d = 0; d < NDIR; ++d) row[d] = 0.5 * st[d];
            row[NDIR] = st[NDIR];
            if (zp == 0) {
                // interior stencil: entries of opposite directions are equal
                // (symmetric element matrices, translation invariance inside
                // the tet); the interior kernel uses one weight per pair
                double mx = 0.0;
                for (int d = 0; d < NDIR; ++d) mx = std::max(mx, std::fabs(row[d]));
                for (int d = 0; d < NDIR / 2; ++d) {
                    if (std::fabs(row[d] - row[d + NDIR / 2]) > 1e-12 * mx)
                        return fail(c, HHG_EMESH, "tet %d: interior stencil is not symmetric", t);
                    row[d] = row[d + NDIR / 2] = 0.5 * (row[d] + row[d + NDIR / 2]);
                }
            }
            // restriction weights: 1/2 per coarse edge split evenly over the
            // tets holding that edge; the centre 1 split over the node's tets
            rw[NDIR] = 1.0 / tp.valence(t, zp);
            for (int d = 0; d < NDIR; ++d) {
                if (!cnt[d]) continue;
                const int zq = zero_pattern(8, ri + DIR[d][0], rj + DIR[d][1], rk + DIR[d][2]);
                rw[d] = 0.5 / tp.valence(t, zp & zq);
            }
        }
    }
    // tensor components D_m = c_m.grad: per tet and kind the half reference
    // entries of each a_m (the same sums as the scalar stencil above)
    {
        static const double CD[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
        L.h_tsten.assign((size_t)tp.nt * 6 * TET_STENCIL, 0.0);
        L.h_temat.assign((size_t)tp.nt * 6 * TET_EMAT, 0.0);
        for (int t = 0; t < tp.nt; ++t)
            for (int m = 0; m < 6; ++m) {
                double E[NTYPE][4][4];
                for (int ty = 0; ty < NTYPE; ++ty) {
                    double p[4][3];
                    for (int a = 0; a < 4; ++a)
                        lattice_point(tp, t, L.n, TYPE_OFF[ty][a][0], TYPE_OFF[ty][a][1], TYPE_OFF[ty][a][2], p[a]);
                    if (!element_matrix_dir(p, CD[m], E[ty])) return fail(c, HHG_EMESH, "tet %d is degenerate", t);
                    for (int a = 0; a < 4; ++a)
                        for (int b = 0; b < 4; ++b)
                            L.h_temat[((size_t)t * 6 + m) * TET_EMAT + ty * 16 + a * 4 + b] = E[ty][a][b] / 4.0;
                }
                for (int zp = 0; zp < 15; ++zp) {
                    if (popcount4(zp) == 4) continue;
                    int ri, rj, rk;
                    representative(zp, ri, rj, rk);
                    double st[NDIR + 1] = {0};
                    for (int ty = 0; ty < NTYPE; ++ty)
                        for (int a = 0; a < 4; ++a) {
                            if (!element_valid(8, ri - TYPE_OFF[ty][a][0], rj - TYPE_OFF[ty][a][1],
                                               rk - TYPE_OFF[ty][a][2], ty))
                                continue;
                            for (int b = 0; b < 4; ++b) {
                                const int d = dir_index(TYPE_OFF[ty][b][0] - TYPE_OFF[ty][a][0],
                                                        TYPE_OFF[ty][b][1] - TYPE_OFF[ty][a][1],
                                                        TYPE_OFF[ty][b][2] - TYPE_OFF[ty][a][2]);
                                st[d] += E[ty][a][b];
                            }
                        }
                    double *row = &L.h_tsten[((size_t)t * 6 + m) * TET_STENCIL + zp * KIND_STRIDE];
                    for (int d = 0; d < NDIR; ++d) row[d] = 0.5 * st[d];
                    row[NDIR] = st[NDIR];
                }
                // the interior rows' pair fields take w_d = w_{d+7}
                const double *w0 = &L.h_tsten[((size_t)t * 6 + m) * TET_STENCIL];
                for (int d = 0; d < NDIR / 2; ++d)
                    if (std::fabs(w0[d] - w0[d + NDIR / 2]) > 1e-12 * (std::fabs(w0[d]) + std::fabs(w0[d + NDIR / 2])))
                        return fail(c, HHG_EMESH, "tet %d: interior stencil of component %d is not point-symmetric",
                                    t, m);
            }
    }
    // nodes on shared primitives: every non-Dirichlet vertex / edge / face of
    // the macro mesh that is not inside one tet, with all tets holding it
    L.h_sh_off.assign(1, 0);
    L.h_sh_copy.clear();
    auto add_node = [&](const std::vector<int> &verts, const std::vector<int> &wts) {
        for (int t = 0; t < tp.nt; ++t) {
            int w[4] = {0, 0, 0, 0};
            int found = 0;
            for (size_t a = 0; a < verts.size(); ++a)
                for (int b = 0; b < 4; ++b)
                    if (tp.tet[4 * t + b] == verts[a]) { w[b] = wts[a]; ++found; }
            if (found != (int)verts.size()) continue;
            const int zp = (w[0] == 0) | ((w[1] == 0) << 1) | ((w[2] == 0) << 2) | ((w[3] == 0) << 3);
            L.h_sh_copy.push_back(pack_copy(t, zp, w[1], w[2], w[3]));
        }
        L.h_sh_off.push_back((int32_t)L.h_sh_copy.size());
    };
    for (int v = 0; v < tp.nv; ++v)
        if (tp.vpos[v] >= 0 && !tp.v_bnd[v]) add_node({v}, {L.n});
    for (size_t e = 0; e < tp.edges.size(); ++e)
        if (!tp.e_bnd[e])
            for (int s = 1; s < L.n; ++s) add_node({tp.edges[e][0], tp.edges[e][1]}, {L.n - s, s});
    for (size_t f = 0; f < tp.faces.size(); ++f)
        if (!tp.f_bnd[f])
            for (int tt = 1; tt < L.n; ++tt)
                for (int s = 1; s + tt < L.n; ++s)
                    add_node({tp.faces[f][0], tp.faces[f][1], tp.faces[f][2]}, {L.n - s - tt, s, tt});
    L.n_shared = (int)L.h_sh_off.size() - 1;

    // order for memory locality: each node's first copy is one in whose tet
    // its primitive runs along the slot order (a k = 0 face, then the face
    // opposite vertex 0), and nodes go by the slot of that copy
    if (L.n_shared > 1) {
        auto rank = [](int kind) { return (kind & 8) ? 0 : (kind & 1) ? 1 : 2; };
        std::vector<int64_t> key(L.n_shared);
        std::vector<uint64_t> first(L.n_shared);
        for (int q = 0; q < L.n_shared; ++q) {
            int best = L.h_sh_off[q], br = 3;
            for (int p = L.h_sh_off[q]; p < L.h_sh_off[q + 1]; ++p) {
                int t, kind, i, j, k;
                unpack_copy(L.h_sh_copy[p], t, kind, i, j, k);
                if (rank(kind) < br) { br = rank(kind); best = p; }
            }
            std::swap(L.h_sh_copy[L.h_sh_off[q]], L.h_sh_copy[best]);
            int t, kind, i, j, k;
            unpack_copy(L.h_sh_copy[L.h_sh_off[q]], t, kind, i, j, k);
            key[q] = (int64_t)t * L.Spad + slot_of(L.n, i, j, k);
        }
        std::vector<int> order(L.n_shared);
        for (int q = 0; q < L.n_shared; ++q) order[q] = q;
        std::sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
        std::vector<int32_t> off2(1, 0);
        std::vector<uint64_t> copy2;
        copy2.reserve(L.h_sh_copy.size());
        for (int q : order) {
            for (int p = L.h_sh_off[q]; p < L.h_sh_off[q + 1]; ++p) copy2.push_back(L.h_sh_copy[p]);
            off2.push_back((int32_t)copy2.size());
        }
        L.h_sh_off.swap(off2);
        L.h_sh_copy.swap(copy2);
    }

    // merged neighbour lists of the shared rows.  An entry is kept for a
    // (copy, direction) when the neighbour lies in the copy's tet and either
    // the tet-restricted scaled weight or some element coupling in that
    // direction is not negligible (below 1e-14 of the tet's largest entry);
    // copies of one neighbour node in different tets (found by its macro
    // vertices and barycentric weights) share an entry.
    if (L.n_shared > 0) {
        std::vector<uint8_t> need((size_t)tp.nt * 16 * NDIR, 0);
        for (int t = 0; t < tp.nt; ++t) {
            double ms = 0.0, me = 0.0;
            for (int q = 0; q < TET_STENCIL; ++q) ms = std::max(ms, std::fabs(L.h_sten[(size_t)t * TET_STENCIL + q]));
            for (int q = 0; q < TET_EMAT; ++q) me = std::max(me, std::fabs(L.h_emat[(size_t)t * TET_EMAT + q]));
            for (int zp = 0; zp < 15; ++zp) {
                if (popcount4(zp) == 4) continue;
                uint8_t *nd = &need[((size_t)t * 16 + zp) * NDIR];
                const double *row = &L.h_sten[(size_t)t * TET_STENCIL + zp * KIND_STRIDE];
                for (int d = 0; d < NDIR; ++d) nd[d] = std::fabs(row[d]) > 1e-14 * ms;
                int ri, rj, rk;
                representative(zp, ri, rj, rk);
                for (int ty = 0; ty < NTYPE; ++ty)
                    for (int a = 0; a < 4; ++a) {
                        if (!element_valid(8, ri - TYPE_OFF[ty][a][0], rj - TYPE_OFF[ty][a][1],
                                           rk - TYPE_OFF[ty][a][2], ty))
                            continue;
                        for (int b = 0; b < 4; ++b) {
                            if (b == a) continue;
                            const int d = dir_index(TYPE_OFF[ty][b][0] - TYPE_OFF[ty][a][0],
                                                    TYPE_OFF[ty][b][1] - TYPE_OFF[ty][a][1],
                                                    TYPE_OFF[ty][b][2] - TYPE_OFF[ty][a][2]);
                            if (std::fabs(L.h_emat[(size_t)t * TET_EMAT + ty * 16 + a * 4 + b]) > 1e-14 * me)
                                nd[d] = 1;
                        }
                    }
            }
        }
        // the scaled operator's own pattern: directions whose tet-restricted
        // scaled weight is not negligible (the element couplings of the
        // nodal form widen the pattern above; on Kuhn meshes the scaled
        // stencil has 6 of the 14 directions)
        std::vector<uint8_t> need_s((size_t)tp.nt * 16 * NDIR, 0);
        for (int t = 0; t < tp.nt; ++t) {
            double ms = 0.0;
            for (int q = 0; q < TET_STENCIL; ++q) ms = std::max(ms, std::fabs(L.h_sten[(size_t)t * TET_STENCIL + q]));
            for (int zp = 0; zp < 15; ++zp) {
                if (popcount4(zp) == 4) continue;
                uint8_t *nd = &need_s[((size_t)t * 16 + zp) * NDIR];
                const double *row = &L.h_sten[(size_t)t * TET_STENCIL + zp * KIND_STRIDE];
                for (int d = 0; d < NDIR; ++d) nd[d] = std::fabs(row[d]) > 1e-14 * ms;
            }
        }
        // the tensor operator's pattern: every component's tet-restricted
        // weights and element matrices (wider than the scalar one where a
        // component couples a direction the scalar stencil does not)
        std::vector<uint8_t> need_t((size_t)tp.nt * 16 * NDIR, 0);
        for (int t = 0; t < tp.nt; ++t) {
            double ms = 0.0, me = 0.0;
            for (int q = 0; q < 6 * TET_STENCIL; ++q)
                ms = std::max(ms, std::fabs(L.h_tsten[(size_t)t * 6 * TET_STENCIL + q]));
            for (int q = 0; q < 6 * TET_EMAT; ++q) me = std::max(me, std::fabs(L.h_temat[(size_t)t * 6 * TET_EMAT + q]));
            for (int zp = 0; zp < 15; ++zp) {
                if (popcount4(zp) == 4) continue;
                uint8_t *nd = &need_t[((size_t)t * 16 + zp) * NDIR];
                for (int m = 0; m < 6; ++m) {
                    const double *row = &L.h_tsten[((size_t)t * 6 + m) * TET_STENCIL + zp * KIND_STRIDE];
                    for (int d = 0; d < NDIR; ++d)
                        if (std::fabs(row[d]) > 1e-14 * ms) nd[d] = 1;
                }
                int ri, rj, rk;
                representative(zp, ri, rj, rk);
                for (int ty = 0; ty < NTYPE; ++ty)
                    for (int a = 0; a < 4; ++a) {
                        if (!element_valid(8, ri - TYPE_OFF[ty][a][0], rj - TYPE_OFF[ty][a][1],
                                           rk - TYPE_OFF[ty][a][2], ty))
                            continue;
                        for (int b = 0; b < 4; ++b) {
                            if (b == a) continue;
                            const int d = dir_index(TYPE_OFF[ty][b][0] - TYPE_OFF[ty][a][0],
                                                    TYPE_OFF[ty][b][1] - TYPE_OFF[ty][a][1],
                                                    TYPE_OFF[ty][b][2] - TYPE_OFF[ty][a][2]);
                            for (int m = 0; m < 6; ++m)
                                if (std::fabs(L.h_temat[((size_t)t * 6 + m) * TET_EMAT + ty * 16 + a * 4 + b]) >
                                    1e-14 * me)
                                    nd[d] = 1;
                        }
                    }
            }
        }
        const int64_t ncopy = (int64_t)L.h_sh_copy.size();
        std::vector<int64_t> hcslot(ncopy), hself(L.n_shared);
        struct Key { int v[4], w[4]; };
        auto key_of = [&](int t, int i, int j, int k, Key &K) {
            const int wt[4] = {L.n - i - j - k, i, j, k};
            int c2 = 0;
            std::pair<int, int> pr[4];
            for (int a = 0; a < 4; ++a)
                if (wt[a] > 0) pr[c2++] = {tp.tet[4 * t + a], wt[a]};
            std::sort(pr, pr + c2);
            for (int a = 0; a < 4; ++a) {
                K.v[a] = a < c2 ? pr[a].first : -1;
                K.w[a] = a < c2 ? pr[a].second : 0;
            }
        };
        auto same = [](const Key &A, const Key &B) {
            for (int a = 0; a < 4; ++a)
                if (A.v[a] != B.v[a] || A.w[a] != B.w[a]) return false;
            return true;
        };
        // one merged pattern per `need`: map[copy][d] = entry, the ELL table of
        // neighbour slots (padding entries = the node itself) and its width
        // merged_scaled: keep only the entries whose merged scaled weight (the
        // sum of the copies' tet-restricted weights onto the entry; the
        // coefficient is that sum times k_q + k_m) is not negligible: on the
        // Kuhn meshes the restricted weights of two tets cancel exactly in 8
        // of a face node's directions, although neither vanishes alone
        auto build_ell = [&](const std::vector<uint8_t> &need, std::vector<int8_t> &hmap, std::vector<int64_t> &ell,
                             int &width, bool merged_scaled = false) -> hhg_status {
            hmap.assign((size_t)ncopy * 16, -1);
            std::vector<int32_t> ecount(L.n_shared);
            std::vector<int64_t> enb;  // entries of all nodes, node after node
            enb.reserve((size_t)L.n_shared * 8);
            width = 0;
            std::vector<Key> keys;
            std::vector<int64_t> slots;
            for (int q = 0; q < L.n_shared; ++q) {
                keys.clear();
                slots.clear();
                for (int p = L.h_sh_off[q]; p < L.h_sh_off[q + 1]; ++p) {
                    int t, kind, i, j, k;
                    unpack_copy(L.h_sh_copy[p], t, kind, i, j, k);
                    hcslot[p] = (int64_t)t * L.Spad + slot_of(L.n, i, j, k);
                    if (p == L.h_sh_off[q]) hself[q] = hcslot[p];
                    const uint8_t *nd = &need[((size_t)t * 16 + kind) * NDIR];
                    for (int d = 0; d < NDIR; ++d) {
                        const int i2 = i + DIR[d][0], j2 = j + DIR[d][1], k2 = k + DIR[d][2];
                        if (!nd[d] || !in_lattice(L.n, i2, j2, k2)) continue;
                        Key K;
                        key_of(t, i2, j2, k2, K);
                        int m = -1;
                        for (size_t e = 0; e < keys.size(); ++e)
                            if (same(keys[e], K)) { m = (int)e; break; }
                        if (m < 0) {
                            m = (int)keys.size();
                            keys.push_back(K);
                            slots.push_back((int64_t)t * L.Spad + slot_of(L.n, i2, j2, k2));
                        }
                        if (m > 127) return fail(c, HHG_EMESH, "shared node with more than 128 neighbours");
                        hmap[(size_t)p * 16 + d] = (int8_t)m;
                    }
                }
                if (merged_scaled) {
                    std::vector<double> wsum(keys.size(), 0.0);
                    double wmax = 0.0;
                    for (int p = L.h_sh_off[q]; p < L.h_sh_off[q + 1]; ++p) {
                        int t, kind, i, j, k;
                        unpack_copy(L.h_sh_copy[p], t, kind, i, j, k);
                        const double *row = &L.h_sten[(size_t)t * TET_STENCIL + kind * KIND_STRIDE];
                        for (int d = 0; d < NDIR; ++d) {
                            wmax = std::max(wmax, std::fabs(row[d]));
                            const int m = hmap[(size_t)p * 16 + d];
                            if (m >= 0) wsum[m] += row[d];
                        }
                    }
                    std::vector<int> remap(keys.size(), -1);
                    std::vector<Key> k2;
                    std::vector<int64_t> s2;
                    for (size_t e = 0; e < keys.size(); ++e)
                        if (std::fabs(wsum[e]) > 1e-12 * wmax) {
                            remap[e] = (int)k2.size();
                            k2.push_back(keys[e]);
                            s2.push_back(slots[e]);
                        }
                    for (int p = L.h_sh_off[q]; p < L.h_sh_off[q + 1]; ++p)
                        for (int d = 0; d < NDIR; ++d) {
                            int8_t &m = hmap[(size_t)p * 16 + d];
                            if (m >= 0) m = (int8_t)remap[m];
                        }
                    keys.swap(k2);
                    slots.swap(s2);
                }
                ecount[q] = (int32_t)keys.size();
                width = std::max(width, (int)keys.size());
                enb.insert(enb.end(), slots.begin(), slots.end());
            }
            ell.assign((size_t)width * L.n_shared, 0);
            int64_t pos = 0;
            for (int q = 0; q < L.n_shared; ++q) {
                for (int m = 0; m < width; ++m)
                    ell[(size_t)m * L.n_shared + q] = m < ecount[q] ? enb[pos + m] : hself[q];
                pos += ecount[q];
            }
            return HHG_OK;
        };
        std::vector<int8_t> hmap, hmap_t, hmap_s;
        std::vector<int64_t> ell, ell_t, ell_s;
        int width = 0, width_t = 0, width_s = 0;
        TRY(build_ell(need, hmap, ell, width));
        TRY(build_ell(need_t, hmap_t, ell_t, width_t));
        TRY(build_ell(need_s, hmap_s, ell_s, width_s, true));
        L.sh_w = width;
        // macro primitive of each shared node from the zero pattern of its
        // barycentric weights: three zero weights = vertex, two = edge, one = face
        L.h_sh_prim.assign((size_t)L.n_shared, 0);
        for (int q = 0; q < L.n_shared; ++q) {
            int t, kind, i, j, k;
            unpack_copy(L.h_sh_copy[L.h_sh_off[q]], t, kind, i, j, k);
            const int zeros = __builtin_popcount((unsigned)kind);
            L.h_sh_prim[q] = (uint8_t)(zeros == 3 ? 1 : zeros == 2 ? 2 : 4);
        }
        {
            std::vector<uint8_t> cp = L.h_sh_prim;
            if (cp.empty()) cp.assign(1, 0);
            TRY(upload(c, &L.sh_prim, cp));
        }
        L.sh_wt = width_t;
        TRY(upload(c, &L.sh_nb, ell));
        TRY(upload(c, &L.sh_nbt, ell_t));
        TRY(upload(c, &L.sh_mapt, hmap_t));
        TRY(upload(c, &L.sh_self, hself));
        TRY(upload(c, &L.sh_cslot, hcslot));
        TRY(upload(c, &L.sh_map, hmap));
        L.sh_ws = width_s;
        TRY(upload(c, &L.sh_nbs, ell_s));
        if ((uint64_t)tp.nt * (uint64_t)L.Spad <= UINT32_MAX) {
            auto narrow = [](const std::vector<int64_t> &a) {
                return std::vector<uint32_t>(a.begin(), a.end());
            };
            TRY(upload(c, &L.sh_nb32, narrow(ell)));
            TRY(upload(c, &L.sh_self32, narrow(hself)));
            TRY(upload(c, &L.sh_cslot32, narrow(hcslot)));
            TRY(upload(c, &L.sh_nbs32, narrow(ell_s)));
        }
        TRY(upload(c, &L.sh_maps, hmap_s));
        {
            const int64_t nes = std::max<int64_t>(1, (int64_t)width_s * L.n_shared);
            TRY(dalloc(c, &L.sh_css64, nes));
            TRY(dalloc(c, &L.sh_css32, nes));
        }
        const int64_t ne = std::max<int64_t>(1, (int64_t)width * L.n_shared);
        TRY(dalloc(c, &L.sh_cs64, ne));
        TRY(dalloc(c, &L.sh_cn64, ne));
        TRY(dalloc(c, &L.sh_cs32, ne));
        TRY(dalloc(c, &L.sh_cn32, ne));
    }

    // column-marching work items: waves over 62 in-plane offsets (plus one
    // halo lane each side) and chunks of kc planes; kc is the largest of
    // 32/16/8/4 that still gives the target wave count over all tets
    {
        const int n = L.n;
        const int64_t T0 = tri_count(n);
        auto diag_of = [](int64_t t) {
            int64_t d = (int64_t)((std::sqrt(8.0 * (double)t + 1.0) - 1.0) / 2.0);
            while ((d + 1) * (d + 2) / 2 <= t) ++d;
            while (d > 0 && d * (d + 1) / 2 > t) --d;
            return d;
        };
        // items for waves of `width` rows: chunk length kc is the largest of
        // 32/16/8/4 that still gives `target` waves over all tets
        auto build_items = [&](int width, int64_t target, std::vector<uint32_t> &out, int &kc_out) {
            std::vector<int> kcs = {32, 16, 8, 4};
            if (const char *e = std::getenv("HHG_MARCH_KC")) {  // tuning override
                const int v = std::atoi(e);
                if (v >= 1 && v <= 1024) kcs = {v};
            }
            for (int kc : kcs) {
                out.clear();
                // k chunks outer, in-plane segments inner: the waves of one
                // block then cover neighbouring diagonals of the same planes
                // and share their loads through the CU's L1
                std::vector<std::pair<int64_t, int>> seg;  // (t0, last interior plane)
                for (int64_t t0 = 0; t0 < T0; t0 += width) {
                    int64_t smin = -1;
                    for (int64_t t = t0; t < std::min<int64_t>(t0 + width, T0); ++t) {
                        const int64_t d = diag_of(t), i = t - d * (d + 1) / 2;
                        if (d >= 2 && d <= n - 2 && i >= 1 && i <= d - 1) { smin = d; break; }
                    }
                    if (smin >= 0) seg.push_back({t0, (int)(n - 1 - smin)});
                }
                for (int k0 = 1; k0 <= n - 3; k0 += kc)
                    for (const auto &sg : seg) {
                        if (k0 > sg.second) continue;
                        const int k1 = std::min(sg.second, k0 + kc - 1);
                        out.push_back((uint32_t)sg.first);
                        out.push_back((uint32_t)k0 | ((uint32_t)k1 << 16));
                    }
                kc_out = kc;
                if ((int64_t)tp.nt * (int64_t)(out.size() / 2) >= target) break;
            }
        };
        // one-row items (FP32 scaled, nodal rows): 4K waves (unit tet level 8:
        // 8-plane chunks instead of 4, FP32 scaled 222 -> 243 GDoF/s; meshes
        // of several tets keep 32)
        build_items(62, 4096, L.h_items, L.kc);
        // two-rows-per-lane items: FP64 prefers more, shorter waves than FP32
        // (a single tet at level 8 gets 8-plane chunks: 2-3% faster than 4)
        build_items(126, tp.nt >= 4 ? 8192 : (int64_t)2048 * tp.nt, L.h_items2, L.kc2);
        L.n_items2 = (int)(L.h_items2.size() / 2);
        build_items(126, 4096, L.h_items2f, L.kc2f);
        L.n_items2f = (int)(L.h_items2f.size() / 2);
        // LDS-staged kernel: blocks of 1008 consecutive offsets (the plane
        // region it stages must fit 1536 elements: n <= 256)
        L.h_itemsL.clear();
        L.n_itemsL = 0;
        if (n >= 4 && n <= 256) {
            build_items(1008, 2048, L.h_itemsL, L.kcL);
            L.n_itemsL = (int)(L.h_itemsL.size() / 2);
        }
        L.n_items = (int)(L.h_items.size() / 2);
        L.h_bnd.clear();
        for (int k = 0; k <= n; ++k)
            for (int sd = 0; sd + k <= n; ++sd)
                for (int i = 0; i <= sd; ++i) {
                    const int zp = zero_pattern(n, i, sd - i, k);
                    if (zp) L.h_bnd.push_back((uint32_t)(slot_of(n, i, sd - i, k) << 4) | (uint32_t)zp);
                }
        L.n_bnd = (int)L.h_bnd.size();
        std::vector<uint32_t> items_copy = L.h_items;
        uint32_t *ip = nullptr;
        TRY(upload(c, &ip, items_copy));
        L.items = (uint2 *)ip;
        {
            std::vector<uint32_t> cp = L.h_itemsL;
            uint32_t *ipl = nullptr;
            if (cp.empty()) cp.assign(2, 0u);
            TRY(upload(c, &ipl, cp));
            L.itemsL = (uint2 *)ipl;
        }
        for (int pr = 0; pr < 2; ++pr) {
            std::vector<uint32_t> cp = pr ? L.h_items2f : L.h_items2;
            uint32_t *ip2 = nullptr;
            if (cp.empty()) cp.assign(2, 0u);  // never read when the count is 0
            TRY(upload(c, &ip2, cp));
            (pr ? L.items2f : L.items2) = (uint2 *)ip2;
        }
        TRY(upload(c, &L.bnd, L.h_bnd));
    }

    std::vector<float> s32(L.h_sten.begin(), L.h_sten.end()), e32(L.h_emat.begin(), L.h_emat.end()),
        r32(L.h_rstw.begin(), L.h_rstw.end());
    TRY(upload(c, &L.sten64, L.h_sten));
    {
        std::vector<float> t32(L.h_tsten.begin(), L.h_tsten.end()), te32(L.h_temat.begin(), L.h_temat.end());
        TRY(upload(c, &L.tsten64, L.h_tsten));
        TRY(upload(c, &L.tsten32, t32));
        TRY(upload(c, &L.temat64, L.h_temat));
        TRY(upload(c, &L.temat32, te32));
    }
    TRY(upload(c, &L.emat64, L.h_emat));
    TRY(upload(c, &L.rstw64, L.h_rstw));
    TRY(upload(c, &L.sten32, s32));
    TRY(upload(c, &L.emat32, e32));
    TRY(upload(c, &L.rstw32, r32));
    TRY(upload(c, &L.dmask, L.h_dmask));
    TRY(upload(c, &L.smask, L.h_smask));
    TRY(upload(c, &L.sh_off, L.h_sh_off));
    TRY(upload(c, &L.sh_copy, L.h_sh_copy));
    // coefficient and work vectors
    TRY(dalloc(c, &L.k64, L.n_slots));
    TRY(dalloc(c, &L.k32, L.n_slots));
    TRY(dalloc(c, &L.invd64, L.n_slots));
    TRY(dalloc(c, &L.invd32, L.n_slots));
    TRY(dalloc(c, &L.r64, L.n_slots));
    TRY(dalloc(c, &L.d64, L.n_slots));
    TRY(dalloc(c, &L.r32, L.n_slots));
    TRY(dalloc(c, &L.d32, L.n_slots));
    TRY(dalloc(c, &L.f32, L.n_slots));
    TRY(dalloc(c, &L.u32, L.n_slots));
    TRY(dalloc(c, &L.logk32, L.n_slots));
    if (l < c->max_level) {
        TRY(dalloc(c, &L.f64, L.n_slots));
        TRY(dalloc(c, &L.u64, L.n_slots));
    }
    // Dirichlet slots of the work vectors must read 0 even before first use
    HIPCHK(c, hipMemset(L.r64, 0, L.n_slots * 8));
    HIPCHK(c, hipMemset(L.r32, 0, L.n_slots * 4));
    HIPCHK(c, hipMemset(L.f32, 0, L.n_slots * 4));
    HIPCHK(c, hipMemset(L.u32, 0, L.n_slots * 4));
    HIPCHK(c, hipMemset(L.d64, 0, L.n_slots * 8));
    HIPCHK(c, hipMemset(L.d32, 0, L.n_slots * 4));
    if (L.f64) HIPCHK(c, hipMemset(L.f64, 0, L.n_slots * 8));
    if (L.u64) HIPCHK(c, hipMemset(L.u64, 0, L.n_slots * 8));
    return HHG_OK;
}

hhg_status ensure_canon_maps(hhg_ctx c, int l)
{
    Level &L = c->lv[l];
    if (L.slot2canon) return HHG_OK;
    if (L.n_nodes >= (int64_t)1 << 31)
        return fail(c, HHG_EINVAL, "level %d has too many nodes for canonical maps", l);
    std::vector<int32_t> s2c((size_t)L.n_slots, -1);
    std::vector<int64_t> c2s((size_t)L.n_nodes, -1);
    const Topology &tp = c->topo;
    for (int t = 0; t < tp.nt; ++t)
        for (int k = 0; k <= L.n; ++k)
            for (int j = 0; j + k <= L.n; ++j)
                for (int i = 0; i + j + k <= L.n; ++i) {
                    const int64_t slot = (int64_t)t * L.Spad + slot_of(L.n, i, j, k);
                    const int64_t ci = canon_index(tp, t, L.n, i, j, k, L.h_poff.data());
                    if (ci < 0 || ci >= L.n_nodes)
                        return fail(c, HHG_EMESH, "canonical numbering out of range at level %d", l);
                    const int zp = zero_pattern(L.n, i, j, k);
                    s2c[slot] = ((L.h_dmask[t] >> zp) & 1) ? (int32_t)(-ci - 1) : (int32_t)ci;
                    if (c2s[ci] < 0) c2s[ci] = slot;
                }
    for (int64_t ci = 0; ci < L.n_nodes; ++ci)
        if (c2s[ci] < 0) return fail(c, HHG_EMESH, "canonical node %lld has no slot", (long long)ci);
    TRY(upload(c, &L.slot2canon, s2c));
    TRY(upload(c, &L.canon2slot, c2s));
    return HHG_OK;
}

// support lists of the geometric coarse coefficients of level l (from level
// l + 1) for the nodes on macro primitives: every distinct fine node f with
// P_fc != 0 (the coincident node, weight 1, and the midpoint of every coarse
// edge at the node, weight 1/2, over all copies; distinct by canonical index)
hhg_status build_coarsen_lists(hhg_ctx c, int l)
{
    Level &Lc = c->lv[l], &Lf = c->lv[l + 1];
    if (Lc.cg_ready) return HHG_OK;
    const Topology &tp = c->topo;
    const int nc = Lc.n, nf = Lf.n;
    struct Copy {
        int64_t ci;
        int t, i, j, k;
    };
    std::vector<Copy> cps;
    for (int t = 0; t < tp.nt; ++t)
        for (int k = 0; k <= nc; ++k)
            for (int j = 0; j + k <= nc; ++j)
                for (int i = 0; i + j + k <= nc; ++i) {
                    if (i > 0 && j > 0 && k > 0 && i + j + k < nc) continue;
                    cps.push_back({canon_index(tp, t, nc, i, j, k, Lc.h_poff.data()), t, i, j, k});
                }
    std::sort(cps.begin(), cps.end(), [](const Copy &a, const Copy &b) {
        return a.ci != b.ci ? a.ci < b.ci : a.t < b.t;
    });
    std::vector<int32_t> off(1, 0), coff(1, 0);
    std::vector<int64_t> fslot, cslot, seen;
    std::vector<double> w;
    for (size_t a = 0; a < cps.size();) {
        size_t b = a;
        while (b < cps.size() && cps[b].ci == cps[a].ci) ++b;
        seen.clear();
        auto add = [&](int t, int fi, int fj, int fk, double wt) {
            const int64_t fci = canon_index(tp, t, nf, fi, fj, fk, Lf.h_poff.data());
            for (int64_t x : seen)
                if (x == fci) return;
            seen.push_back(fci);
            fslot.push_back((int64_t)t * Lf.Spad + slot_of(nf, fi, fj, fk));
            w.push_back(wt);
        };
        for (size_t q = a; q < b; ++q) {
            const Copy &C = cps[q];
            add(C.t, 2 * C.i, 2 * C.j, 2 * C.k, 1.0);
            for (int d = 0; d < NDIR; ++d) {
                const int i2 = C.i + DIR[d][0], j2 = C.j + DIR[d][1], k2 = C.k + DIR[d][2];
                if (!in_lattice(nc, i2, j2, k2)) continue;
                add(C.t, 2 * C.i + DIR[d][0], 2 * C.j + DIR[d][1], 2 * C.k + DIR[d][2], 0.5);
            }
            cslot.push_back((int64_t)C.t * Lc.Spad + slot_of(nc, C.i, C.j, C.k));
        }
        off.push_back((int32_t)fslot.size());
        coff.push_back((int32_t)cslot.size());
        a = b;
    }
    Lc.cg_n = (int)(off.size() - 1);
    TRY(upload(c, &Lc.cg_off, off));
    TRY(upload(c, &Lc.cg_coff, coff));
    TRY(upload(c, &Lc.cg_fslot, fslot.empty() ? std::vector<int64_t>(1, 0) : fslot));
    TRY(upload(c, &Lc.cg_w, w.empty() ? std::vector<double>(1, 0.0) : w));
    TRY(upload(c, &Lc.cg_cslot, cslot.empty() ? std::vector<int64_t>(1, 0) : cslot));
    Lc.cg_ready = true;
    return HHG_OK;
}

// ---------------------------------------------------------------- operator drivers
template <typename T>
hhg_status apply_scaled_t(hhg_ctx c, int l, const T *u, T *y, hipStream_t st)
{
    LevelView<T> V = view<T>(c, l);
    if (c->timing) {
        // an event pair spanning this apply's stencil kernels, stamped by the
        // launches themselves (events pooled; the pool grows on the first
        // timed applies).  A level without stencil kernels records an empty
        // window.
        const size_t q = 2 * c->tev_used;
        while (c->tev.size() < q + 2) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->tev.push_back(e);
        }
        set_launch_events(c->tev[q], c->tev[q + 1]);
        const hipError_t e = launch_scaled<T>(V, MODE_APPLY, u, nullptr, y, nullptr, nullptr, st);
        const bool none = launch_events_unused();
        set_launch_events(nullptr, nullptr);
        HIPCHK(c, e);
        if (none) {
            HIPCHK(c, hipEventRecord(c->tev[q], st));
            HIPCHK(c, hipEventRecord(c->tev[q + 1], st));
        }
        ++c->tev_used;
    } else {
        HIPCHK(c, launch_scaled<T>(V, MODE_APPLY, u, nullptr, y, nullptr, nullptr, st));
    }
    HIPCHK(c, launch_correction<T>(V, corr<T>(c, l), MODE_APPLY, u, y, nullptr, st));
    return HHG_OK;
}

// r = f - A u; if norm, the Euclidean norm over the unknowns (synchronises).
// The norm's per-block partials and the reduced value go to partial_buf and
// scalar_buf when given (device memory the caller provides), else to the
// context's buffers.
template <typename T>
hhg_status residual_t(hhg_ctx c, int l, const T *f, const T *u, T *r, double *norm, hipStream_t st,
                      double *partial_buf = nullptr, double *scalar_buf = nullptr)
{
    LevelView<T> V = view<T>(c, l);
    double *const partial = partial_buf ? partial_buf : c->partial;
    double *const dscalar = scalar_buf ? scalar_buf : c->dscalar;
    int np = 0;
    if (c->op == 1 || c->op == 2) {
        // a tensor form (its partial count was checked against the buffer
        // when its solver state was built)
        HIPCHK(c, launch_tensor<T>(V, c->op - 1, MODE_RESID, u, f, r, partial, &np, st));
    } else if (c->op == 3 || c->op == 4) {
        // the scalar nodal or primitive-mixed form (the scaled residual's grids)
        HIPCHK(c, launch_scalar_form<T>(V, corr<T>(c, l), c->op - 2, MODE_RESID, c->mix_mask, u, f, r, partial,
                                        &np, st));
    } else {
        HIPCHK(c, launch_scaled<T>(V, MODE_RESID, u, f, r, partial, &np, st));
        CorrView<T> C = corr<T>(c, l);
        HIPCHK(c, launch_correction<T>(V, C, MODE_RESID, u, r, partial + np, st));
        if (C.n_rows) np += (C.n_rows + BLOCK - 1) / BLOCK;
    }
    if (norm) {
        HIPCHK(c, launch_reduce(partial, np, 0, dscalar, st));
        HIPCHK(c, hipMemcpyAsync(c->hscalar, dscalar, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        // a NaN sum stays NaN (std::max would turn it into 0, a converged solve)
        const double v = c->hscalar[0];
        *norm = std::isnan(v) ? v : std::sqrt(std::max(0.0, v));
    }
    return HHG_OK;
}

template <typename T> T *oinvd(Level &L, int q);
template <> double *oinvd<double>(Level &L, int q) { return L.oinvd64[q]; }
template <> float *oinvd<float>(Level &L, int q) { return L.oinvd32[q]; }

// smoothing with an operator other than the scaled one: Jacobi, or the
// Chebyshev iteration of the scaled operator (same interval from the
// operator's own bound) as residual plus update passes
template <typename T>
hhg_status smooth_other_t(hhg_ctx c, int l, hhg_smoother sm, int sweeps, double omega, const T *f, T *u,
                          hipStream_t st)
{
    Level &L = c->lv[l];
    const int form = c->op - 1;
    T *r = work_r<T>(L), *d = work_d<T>(L);
    const T *id = oinvd<T>(L, form);
    if (sm == HHG_JACOBI) {
        for (int s = 0; s < sweeps; ++s) {
            TRY(residual_t<T>(c, l, f, u, r, nullptr, st));
            HIPCHK(c, launch_jacobi_update<T>(u, r, id, (T)omega, L.n_slots, st));
        }
        return HHG_OK;
    }
    const double a = 0.1 * L.olam[form], b = L.olam[form];
    const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
    double rho = 1.0 / sigma;
    if (c->op == 4) {
        // the mixed form: fused sweeps as for the scaled operator (the
        // iterate alternates between u and r)
        const LevelView<T> V = view<T>(c, l);
        const CorrView<T> C = corr<T>(c, l);
        T *cur = u, *nxt = r;
        for (int s = 0; s < sweeps; ++s) {
            ChebArgs<T> cb;
            cb.d = d;
            cb.invd = id;
            if (s == 0) {
                cb.first = 1;
                cb.c_r = (T)(1.0 / theta);
            } else {
                const double rn = 1.0 / (2.0 * sigma - rho);
                cb.c_old = (T)(rn * rho);
                cb.c_r = (T)(2.0 * rn / delta);
                rho = rn;
            }
            HIPCHK(c, launch_cheb_sweep_mixed<T>(V, C, c->mix_mask, cur, f, nxt, cb, st));
            std::swap(cur, nxt);
        }
        if (cur != u)
            HIPCHK(c, hipMemcpyAsync(u, cur, L.n_slots * sizeof(T), hipMemcpyDeviceToDevice, st));
        return HHG_OK;
    }
    for (int s = 0; s < sweeps; ++s) {
        T c_old = T(0), c_r = (T)(1.0 / theta);
        if (s > 0) {
            const double rn = 1.0 / (2.0 * sigma - rho);
            c_old = (T)(rn * rho);
            c_r = (T)(2.0 * rn / delta);
            rho = rn;
        }
        TRY(residual_t<T>(c, l, f, u, r, nullptr, st));
        HIPCHK(c, launch_cheb_update<T>(u, d, r, id, c_old, c_r, L.n_slots, st));
    }
    return HHG_OK;
}

template <typename T>
hhg_status smooth_t(hhg_ctx c, int l, hhg_smoother sm, int sweeps, double omega, const T *f, T *u,
                    hipStream_t st)
{
    if (c->op) return smooth_other_t<T>(c, l, sm, sweeps, omega, f, u, st);
    Level &L = c->lv[l];
    T *r = work_r<T>(L), *d = work_d<T>(L);
    const T *id = invd<T>(L);
    if (sm == HHG_JACOBI) {
        for (int s = 0; s < sweeps; ++s) {
            TRY(residual_t<T>(c, l, f, u, r, nullptr, st));
            HIPCHK(c, launch_jacobi_update<T>(u, r, id, (T)omega, L.n_slots, st));
        }
        return HHG_OK;
    }
    // Chebyshev iteration on D^{-1} A over [0.1, 1] x lambda_max.  Each sweep
    // is one fused pass (residual, direction and next iterate together): the
    // iterate alternates between u and the level's residual vector, which
    // the smoother does not otherwise need; an odd sweep count copies back.
    const double a = 0.1 * L.lam, b = L.lam;
    const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
    double rho = 1.0 / sigma;
    const LevelView<T> V = view<T>(c, l);
    const CorrView<T> C = corr<T>(c, l);
    T *cur = u, *nxt = r;
    for (int s = 0; s < sweeps; ++s) {
        ChebArgs<T> cb;
        cb.d = d;
        cb.invd = id;
        if (s == 0) {
            cb.first = 1;
            cb.c_r = (T)(1.0 / theta);
        } else {
            const double rn = 1.0 / (2.0 * sigma - rho);
            cb.c_old = (T)(rn * rho);
            cb.c_r = (T)(2.0 * rn / delta);
            rho = rn;
        }
        HIPCHK(c, launch_cheb_sweep<T>(V, C, cur, f, nxt, cb, st));
        std::swap(cur, nxt);
    }
    if (cur != u)
        HIPCHK(c, hipMemcpyAsync(u, cur, L.n_slots * sizeof(T), hipMemcpyDeviceToDevice, st));
    return HHG_OK;
}

template <typename T>
hhg_status coarse_solve_t(hhg_ctx c, const T *f, T *u, hipStream_t st)
{
    Level &L = c->lv[c->coarse];
    const CoarseInv &C = c->co[c->op];
    HIPCHK(c, launch_fill<T>(u, T(0), L.n_slots, st));
    HIPCHK(c, launch_coarse_solve<T>(C.ainv, C.cu, C.cgather, C.ccoff, C.ccslot, f, u, C.cf, st));
    return HHG_OK;
}

template <typename T>
hhg_status learned_smooth_t(hhg_ctx c, int l, int sweeps, const T *f, T *u, hipStream_t st);

// V(pre,post) cycle; the learned smoother (if asked for) acts on the cycle's
// top level only, coarser levels use Chebyshev
template <typename T>
hhg_status vcycle_t(hhg_ctx c, int l, const T *f, T *u, int pre, int post, hhg_smoother sm,
                    hipStream_t st)
{
    if (l == c->coarse) return coarse_solve_t<T>(c, f, u, st);
    Level &L = c->lv[l], &Lc = c->lv[l - 1];
    const hhg_smoother below = sm == HHG_LEARNED ? HHG_CHEBYSHEV : sm;
    if (sm == HHG_LEARNED) TRY(learned_smooth_t<T>(c, l, pre, f, u, st));
    else TRY(smooth_t<T>(c, l, sm, pre, 2.0 / 3.0, f, u, st));
    T *r = work_r<T>(L);
    TRY(residual_t<T>(c, l, f, u, r, nullptr, st));
    T *fc = work_f<T>(Lc), *uc = work_u<T>(Lc);
    HIPCHK(c, launch_restrict<T>(view<T>(c, l - 1), view<T>(c, l), r, fc, st));
    // the coarse correction starts from zero (the coarse solve overwrites it)
    if (l - 1 > c->coarse) HIPCHK(c, launch_fill<T>(uc, T(0), Lc.n_slots, st));
    TRY(vcycle_t<T>(c, l - 1, fc, uc, pre, post, below, st));
    HIPCHK(c, launch_prolong_add<T>(view<T>(c, l - 1), view<T>(c, l), uc, u, st));
    if (sm == HHG_LEARNED) TRY(learned_smooth_t<T>(c, l, post, f, u, st));
    else TRY(smooth_t<T>(c, l, sm, post, 2.0 / 3.0, f, u, st));
    return HHG_OK;
}

void clear_graphs(hhg_ctx c)
{
    for (auto &kv : c->gcache) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    c->gcache.clear();
}

// one V-cycle of a solve loop: captured once per key into a HIP graph on the
// context's own stream, then replayed (ordered after the caller's stream by
// events, and the caller's stream after it).  The learned smoother's cycles
// (lazy scratch allocation) and a disabled context run eagerly.
template <typename T>
hhg_status vcycle_run(hhg_ctx c, int l, const T *f, T *u, int pre, int post, hhg_smoother sm, hipStream_t st)
{
    if (!c->graphs || sm == HHG_LEARNED) return vcycle_t<T>(c, l, f, u, pre, post, sm, st);
    if (!c->gstream) {
        HIPCHK(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
        for (hipEvent_t &e : c->gev) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    const hhg_ctx_s::GraphKey K{l, pre, post, (int)sm, c->op, c->mix_mask, (int)sizeof(T), march_variant_now(),
                                f, u, c->graph_epoch};
    auto it = c->gcache.find(K);
    if (it == c->gcache.end()) {
        if (c->gcache.size() >= 32) clear_graphs(c);
        for (auto q = c->gcache.begin(); q != c->gcache.end();) {
            if (q->first.epoch != c->graph_epoch) {
                (void)hipGraphExecDestroy(q->second.second);
                (void)hipGraphDestroy(q->second.first);
                q = c->gcache.erase(q);
            } else {
                ++q;
            }
        }
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        HIPCHK(c, hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
        const hhg_status s = vcycle_t<T>(c, l, f, u, pre, post, sm, c->gstream);
        const hipError_t e = hipStreamEndCapture(c->gstream, &g);
        if (s != HHG_OK) {
            if (e == hipSuccess && g) (void)hipGraphDestroy(g);
            return s;
        }
        HIPCHK(c, e);
        const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(c, HHG_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
        }
        it = c->gcache.emplace(K, std::make_pair(g, ge)).first;
    }
    HIPCHK(c, hipEventRecord(c->gev[0], st));
    HIPCHK(c, hipStreamWaitEvent(c->gstream, c->gev[0], 0));
    HIPCHK(c, hipGraphLaunch(it->second.second, c->gstream));
    HIPCHK(c, hipEventRecord(c->gev[1], c->gstream));
    HIPCHK(c, hipStreamWaitEvent(st, c->gev[1], 0));
    return HHG_OK;
}

// ---------------------------------------------------------------- coefficient set-up
// modification (Sec. 4.1, read for 3D): per tet, per edge with a positive
// element entry, compare k_e with the minimum edge average over the edge's
// element patch; replace k_e where triggered.  Builds the correction lists.
hhg_status build_modification(hhg_ctx c, int l)
{
    Level &L = c->lv[l];
    const Topology &tp = c->topo;
    L.n_corr_rows = 0;
    L.n_corr = 0;
    if (c->flags & HHG_FLAG_NO_MODIFICATION) return HHG_OK;
    init_edge_use();
    std::vector<double> kh;  // host copy of k at this level, fetched on demand
    struct Corr {
        int64_t self, nb;
        double delta, base;
        uint8_t nbdir;
    };
    std::map<int64_t, std::vector<Corr>> rows;  // row key -> corrections
    // row key: interior slot -> global slot; shared node q -> -(q+1)
    std::unordered_map<int64_t, int64_t> shared_of;
    bool shared_built = false;
    for (int t = 0; t < tp.nt; ++t) {
        double E[NTYPE][4][4];
        type_matrices(tp, t, L.n, E);
        bool any_pos = false;
        for (int ty = 0; ty < NTYPE; ++ty)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    if (a != b && E[ty][a][b] > 0.0) any_pos = true;
        if (!any_pos) continue;
        double lamT = 1e300;
        for (int ty = 0; ty < NTYPE; ++ty) lamT = std::min(lamT, lambda_min_element(E[ty]));
        if (kh.empty()) {
            kh.resize((size_t)L.n_slots);
            HIPCHK(c, hipMemcpy(kh.data(), L.k64, L.n_slots * sizeof(double), hipMemcpyDeviceToHost));
        }
        if (!shared_built) {
            for (int q = 0; q < L.n_shared; ++q)
                for (int p = L.h_sh_off[q]; p < L.h_sh_off[q + 1]; ++p) {
                    int tt, kind, i, j, k;
                    unpack_copy(L.h_sh_copy[p], tt, kind, i, j, k);
                    shared_of[(int64_t)tt * L.Spad + slot_of(L.n, i, j, k)] = q;
                }
            shared_built = true;
        }
        const double *kt = kh.data() + (int64_t)t * L.Spad;
        auto kat = [&](int i, int j, int k) { return kt[slot_of(L.n, i, j, k)]; };
        const int n = L.n;
        for (int k = 0; k <= n; ++k)
            for (int j = 0; j + k <= n; ++j)
                for (int i = 0; i + j + k <= n; ++i)
                    for (int d = 0; d < 7; ++d) {
                        const int i2 = i + DIR[d][0], j2 = j + DIR[d][1], k2 = k + DIR[d][2];
                        if (!in_lattice(n, i2, j2, k2)) continue;
                        double aplus = -1e300, ref = 0.0, kmin = 1e300;
                        int nel = 0;
                        for (const EdgeUse &eu : g_edge_use[d]) {
                            const int bi = i - TYPE_OFF[eu.t][eu.a][0], bj = j - TYPE_OFF[eu.t][eu.a][1],
                                      bk = k - TYPE_OFF[eu.t][eu.a][2];
                            if (!element_valid(n, bi, bj, bk, eu.t)) continue;
                            ++nel;
                            const double e = E[eu.t][eu.a][eu.b];
                            aplus = std::max(aplus, e);
                            ref += e;
                            double kv[4];
                            for (int v = 0; v < 4; ++v)
                                kv[v] = kat(bi + TYPE_OFF[eu.t][v][0], bj + TYPE_OFF[eu.t][v][1],
                                            bk + TYPE_OFF[eu.t][v][2]);
                            for (int a = 0; a < 4; ++a)
                                for (int b = a + 1; b < 4; ++b) kmin = std::min(kmin, 0.5 * (kv[a] + kv[b]));
                        }
                        if (!nel || !(aplus > 0.0)) continue;
                        const double ka = kat(i, j, k), kb = kat(i2, j2, k2);
                        const double ke = 0.5 * (ka + kb);
                        if (!((ke - kmin) * aplus > kmin * lamT)) continue;
                        const double kmod = kmin * (1.0 + lamT / aplus);
                        const double delta = (kmod - ke) * ref, base = ke * ref;
                        const int64_t sa = (int64_t)t * L.Spad + slot_of(n, i, j, k);
                        const int64_t sb = (int64_t)t * L.Spad + slot_of(n, i2, j2, k2);
                        const bool da = (L.h_dmask[t] >> zero_pattern(n, i, j, k)) & 1;
                        const bool db = (L.h_dmask[t] >> zero_pattern(n, i2, j2, k2)) & 1;
                        auto key = [&](int64_t slot, int zp) -> int64_t {
                            if (zp == 0) return slot;
                            return -(shared_of.at(slot) + 1);
                        };
                        if (!da) rows[key(sa, zero_pattern(n, i, j, k))].push_back({sa, sb, delta, base, (uint8_t)db});
                        if (!db) rows[key(sb, zero_pattern(n, i2, j2, k2))].push_back({sb, sa, delta, base, (uint8_t)da});
                        L.n_corr++;
                    }
    }
    if (rows.empty()) return HHG_OK;
    std::vector<int32_t> coff(1, 0), poff(1, 0);
    std::vector<int64_t> cself, cnb, pslot;
    std::vector<double> cd, cbase;
    std::vector<float> cd32;
    std::vector<uint8_t> cnbd, cprim;
    for (auto &kv : rows) {
        cprim.push_back(kv.first >= 0 ? (uint8_t)0 : L.h_sh_prim[(size_t)(-kv.first - 1)]);
        for (const Corr &q : kv.second) {
            cself.push_back(q.self); cnb.push_back(q.nb); cd.push_back(q.delta);
            cd32.push_back((float)q.delta); cbase.push_back(q.base); cnbd.push_back(q.nbdir);
        }
        coff.push_back((int32_t)cself.size());
        if (kv.first >= 0) {
            pslot.push_back(kv.first);
        } else {
            const int q = (int)(-kv.first - 1);
            for (int p = L.h_sh_off[q]; p < L.h_sh_off[q + 1]; ++p) {
                int tt, kind, i, j, k;
                unpack_copy(L.h_sh_copy[p], tt, kind, i, j, k);
                pslot.push_back((int64_t)tt * L.Spad + slot_of(L.n, i, j, k));
            }
        }
        poff.push_back((int32_t)pslot.size());
    }
    L.n_corr_rows = (int)rows.size();
    TRY(upload(c, &L.c_off, coff));
    TRY(upload(c, &L.p_off, poff));
    TRY(upload(c, &L.c_self, cself));
    TRY(upload(c, &L.c_nb, cnb));
    TRY(upload(c, &L.p_slot, pslot));
    TRY(upload(c, &L.c_prim, cprim));
    TRY(upload(c, &L.c_d64, cd));
    TRY(upload(c, &L.c_d32, cd32));
    TRY(upload(c, &L.c_base, cbase));
    TRY(upload(c, &L.c_nbdir, cnbd));
    return HHG_OK;
}

// Jacobi diagonal (with corrections) and the Gershgorin bound of D^{-1}A
hhg_status build_diag(hhg_ctx c, int l, hipStream_t st)
{
    Level &L = c->lv[l];
    LevelView<double> V = view<double>(c, l);
    const bool corrected = L.n_corr_rows > 0;
    double *asum = nullptr;
    if (corrected) TRY(dalloc(c, &asum, L.n_slots));
    double *gabs = nullptr;
    TRY(dalloc(c, &gabs, 2 * (int64_t)std::max(1, L.n_shared)));
    int np = 0;
    HIPCHK(c, launch_diag<double>(V, L.invd64, asum, c->partial, gabs, &np, st));
    HIPCHK(c, launch_reduce(c->partial, np, 1, c->dscalar, st));
    HIPCHK(c, hipMemcpyAsync(c->hscalar, c->dscalar, sizeof(double), hipMemcpyDeviceToHost, st));
    std::vector<double> g((size_t)2 * L.n_shared);
    if (L.n_shared)
        HIPCHK(c, hipMemcpyAsync(g.data(), gabs, g.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    double lam = c->hscalar[0];
    for (int q = 0; q < L.n_shared; ++q) lam = std::max(lam, 1.0 + g[2 * q] / g[2 * q + 1]);
    if (corrected) {
        // download D and |row| sums, apply the corrections per unique row, upload D
        std::vector<double> D((size_t)L.n_slots), A((size_t)L.n_slots);
        HIPCHK(c, hipMemcpy(D.data(), L.invd64, L.n_slots * 8, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(A.data(), asum, L.n_slots * 8, hipMemcpyDeviceToHost));
        std::vector<int32_t> coff(L.n_corr_rows + 1), poff(L.n_corr_rows + 1);
        HIPCHK(c, hipMemcpy(coff.data(), L.c_off, coff.size() * 4, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(poff.data(), L.p_off, poff.size() * 4, hipMemcpyDeviceToHost));
        const int64_t ncorr = coff.back(), npos = poff.back();
        std::vector<double> cd(ncorr), cb(ncorr);
        std::vector<uint8_t> cn(ncorr);
        std::vector<int64_t> ps(npos);
        HIPCHK(c, hipMemcpy(cd.data(), L.c_d64, ncorr * 8, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(cb.data(), L.c_base, ncorr * 8, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(cn.data(), L.c_nbdir, ncorr, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(ps.data(), L.p_slot, npos * 8, hipMemcpyDeviceToHost));
        std::vector<uint8_t> corrected_slot((size_t)L.n_slots, 0);
        for (int q = 0; q < L.n_corr_rows; ++q) {
            double dd = D[ps[poff[q]]], aa = A[ps[poff[q]]];
            for (int64_t x = coff[q]; x < coff[q + 1]; ++x) {
                dd -= cd[x];
                if (!cn[x]) aa += std::fabs(cb[x] + cd[x]) - std::fabs(cb[x]);
            }
            for (int p = poff[q]; p < poff[q + 1]; ++p) {
                D[ps[p]] = dd;
                A[ps[p]] = aa;
                corrected_slot[ps[p]] = 1;
            }
        }
        HIPCHK(c, hipMemcpy(L.invd64, D.data(), L.n_slots * 8, hipMemcpyHostToDevice));
        // exact maximum over all unknown rows
        lam = 0.0;
        const Topology &tp = c->topo;
        for (int t = 0; t < tp.nt; ++t)
            for (int k = 0; k <= L.n; ++k)
                for (int j = 0; j + k <= L.n; ++j)
                    for (int i = 0; i + j + k <= L.n; ++i) {
                        const int zp = zero_pattern(L.n, i, j, k);
                        if ((L.h_dmask[t] >> zp) & 1) continue;
                        const int64_t s = (int64_t)t * L.Spad + slot_of(L.n, i, j, k);
                        lam = std::max(lam, 1.0 + A[s] / D[s]);
                    }
    }
    L.lam = lam;
    HIPCHK(c, launch_invert_diag<double>(L.invd64, L.n_slots, st));
    HIPCHK(c, launch_convert<double, float>(L.invd64, L.invd32, L.n_slots, st));
    HIPCHK(c, hipStreamSynchronize(st));
    dfree(c, asum);
    dfree(c, gabs);
    return HHG_OK;
}

// dense inverse of the coarse operator (op as hhg_ctx_s::op) over its
// unknowns, column by column from the FP64 apply kernel
hhg_status build_coarse(hhg_ctx c, hipStream_t st, int op = 0)
{
    TRY(ensure_canon_maps(c, c->coarse));
    Level &L = c->lv[c->coarse];
    const Topology &tp = c->topo;
    // unknowns of the coarse level with all their copies, canonical order
    std::vector<std::vector<int64_t>> copies((size_t)L.n_nodes);
    std::vector<uint8_t> dir((size_t)L.n_nodes, 0);
    for (int t = 0; t < tp.nt; ++t)
        for (int k = 0; k <= L.n; ++k)
            for (int j = 0; j + k <= L.n; ++j)
                for (int i = 0; i + j + k <= L.n; ++i) {
                    const int64_t ci = canon_index(tp, t, L.n, i, j, k, L.h_poff.data());
                    copies[ci].push_back((int64_t)t * L.Spad + slot_of(L.n, i, j, k));
                    if ((L.h_dmask[t] >> zero_pattern(L.n, i, j, k)) & 1) dir[ci] = 1;
                }
    std::vector<int64_t> gather, cslot;
    std::vector<int32_t> coff(1, 0);
    for (int64_t ci = 0; ci < L.n_nodes; ++ci) {
        if (dir[ci]) continue;
        gather.push_back(copies[ci][0]);
        for (int64_t s : copies[ci]) cslot.push_back(s);
        coff.push_back((int32_t)cslot.size());
    }
    const int nu = (int)gather.size();
    if (nu == 0) return fail(c, HHG_EINVAL, "coarse level %d has no unknowns", c->coarse);
    if (nu > 4096) return fail(c, HHG_EINVAL, "coarse level %d has %d unknowns (max 4096)", c->coarse, nu);
    std::vector<double> A((size_t)nu * nu);
    std::vector<double> e((size_t)L.n_slots), y((size_t)L.n_slots);
    double *de = L.r64, *dy = L.d64;  // scratch at set-up time
    for (int col = 0; col < nu; ++col) {
        std::fill(e.begin(), e.end(), 0.0);
        for (int p = coff[col]; p < coff[col + 1]; ++p) e[cslot[p]] = 1.0;
        HIPCHK(c, hipMemcpyAsync(de, e.data(), L.n_slots * 8, hipMemcpyHostToDevice, st));
        if (op == 0) TRY(apply_scaled_t<double>(c, c->coarse, de, dy, st));
        else if (op <= 2)
            HIPCHK(c, launch_tensor<double>(view<double>(c, c->coarse), op - 1, MODE_APPLY, de, nullptr, dy, nullptr,
                                            nullptr, st));
        else
            HIPCHK(c, launch_scalar_form<double>(view<double>(c, c->coarse), corr<double>(c, c->coarse), op - 2,
                                                 MODE_APPLY, c->mix_mask, de, nullptr, dy, nullptr, nullptr, st));
        HIPCHK(c, hipMemcpyAsync(y.data(), dy, L.n_slots * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        for (int row = 0; row < nu; ++row) A[(size_t)row * nu + col] = y[gather[row]];
    }
    HIPCHK(c, hipMemsetAsync(de, 0, L.n_slots * 8, st));
    HIPCHK(c, hipMemsetAsync(dy, 0, L.n_slots * 8, st));
    CoarseInv &C = c->co[op];
    if (C.ainv) {
        for (void *p : {(void *)C.ainv, (void *)C.cgather, (void *)C.ccoff, (void *)C.ccslot, (void *)C.cf})
            dfree(c, p);
        C = CoarseInv();
    }
    C.cu = nu;
    if (nu <= 512) {
        if (!invert_dense(A, nu)) return fail(c, HHG_ECOEF, "coarse operator is singular");
        TRY(upload(c, &C.ainv, A));
    } else {
        // larger coarse levels: Gauss-Jordan on the device ([A | I] uploaded
        // once, the inverse extracted into C.ainv)
        std::vector<double> W((size_t)nu * 2 * nu, 0.0);
        for (int r = 0; r < nu; ++r) {
            std::copy(&A[(size_t)r * nu], &A[(size_t)r * nu] + nu, &W[(size_t)r * 2 * nu]);
            W[(size_t)r * 2 * nu + nu + r] = 1.0;
        }
        double *dw = nullptr, *dscr = nullptr;
        int *iscr = nullptr;
        TRY(upload(c, &dw, W));
        TRY(dalloc(c, &dscr, nu + 1));
        TRY(dalloc(c, &iscr, 2));
        TRY(dalloc(c, &C.ainv, (int64_t)nu * nu));
        HIPCHK(c, hipMemsetAsync(iscr, 0, 2 * sizeof(int), st));
        HIPCHK(c, launch_dense_inverse(dw, nu, C.ainv, iscr, dscr, st));
        int sing[2] = {0, 0};
        HIPCHK(c, hipMemcpyAsync(sing, iscr, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        dfree(c, dw);
        dfree(c, dscr);
        dfree(c, iscr);
        if (sing[1]) return fail(c, HHG_ECOEF, "coarse operator is singular");
    }
    TRY(upload(c, &C.cgather, gather));
    TRY(upload(c, &C.ccoff, coff));
    TRY(upload(c, &C.ccslot, cslot));
    TRY(dalloc(c, &C.cf, std::max(nu, 1)));
    HIPCHK(c, hipStreamSynchronize(st));
    return HHG_OK;
}

int default_coarse(hhg_ctx c)
{
    // deep hierarchies: the largest level with at most 4096 unknowns when it
    // lies at least four levels below the finest (its dense inverse is built
    // on the device and costs a few tens of microseconds per cycle, and a
    // deeper exact solve contracts much better on rough coefficients);
    // otherwise the largest with at most 1000
    int deep = -1;
    for (int l = 0; l <= c->max_level; ++l)
        if (c->lv[l].n_unknowns >= 1 && c->lv[l].n_unknowns <= 4096) deep = l;
    if (deep >= 0 && c->max_level - deep >= 4) return deep;
    int best = -1;
    for (int l = 0; l <= c->max_level; ++l)
        if (c->lv[l].n_unknowns >= 1 && c->lv[l].n_unknowns <= 1000) best = l;
    if (best < 0)
        for (int l = 0; l <= c->max_level; ++l)
            if (c->lv[l].n_unknowns >= 1) { best = l; break; }
    return best < 0 ? c->max_level : best;
}

// FP32 scratch vectors of a level for the learned correction
hhg_status learned_scratch(hhg_ctx c, int l)
{
    Level &L = c->lv[l];
    for (float *&p : L.lt)
        if (!p) TRY(dalloc(c, &p, L.n_slots));
    return HHG_OK;
}

// ownership mask: 1 on interior slots and on the first copy of every shared
// non-Dirichlet node (dot products count each unknown once)
hhg_status ensure_own(hhg_ctx c, int l)
{
    Level &L = c->lv[l];
    if (L.own) return HHG_OK;
    std::vector<uint8_t> own((size_t)L.n_slots, 0);
    for (int t = 0; t < c->topo.nt; ++t)
        for (int k = 1; k < L.n; ++k)
            for (int sd = 2; sd + k < L.n; ++sd)
                for (int i = 1; i < sd; ++i) own[(int64_t)t * L.Spad + slot_of(L.n, i, sd - i, k)] = 1;
    for (int q = 0; q < L.n_shared; ++q) {
        int tt, kind, i, j, k;
        unpack_copy(L.h_sh_copy[L.h_sh_off[q]], tt, kind, i, j, k);
        own[(int64_t)tt * L.Spad + slot_of(L.n, i, j, k)] = 1;
    }
    TRY(upload(c, &L.own, own));
    return HHG_OK;
}

double dot_owned(hhg_ctx c, int l, const float *a, const float *b, hipStream_t st, hhg_status *err)
{
    Level &L = c->lv[l];
    int nb = 0;
    *err = HHG_OK;
    if (launch_dot_owned(a, b, L.own, L.n_slots, c->partial, &nb, st) != hipSuccess ||
        launch_reduce(c->partial, nb, 0, c->dscalar, st) != hipSuccess ||
        hipMemcpyAsync(c->hscalar, c->dscalar, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        *err = fail(c, HHG_EHIP, "dot product failed");
        return 0.0;
    }
    return c->hscalar[0];
}

// learned smoothing steps: r = f - A u; u += D^{-1}(omega r + s c(r, k))
template <typename T>
hhg_status learned_smooth_t(hhg_ctx c, int l, int sweeps, const T *f, T *u, hipStream_t st);

template <>
hhg_status learned_smooth_t<double>(hhg_ctx c, int, int, const double *, double *, hipStream_t)
{
    return fail(c, HHG_EINVAL, "the learned smoother runs in FP32");
}

template <>
hhg_status learned_smooth_t<float>(hhg_ctx c, int l, int sweeps, const float *f, float *u, hipStream_t st)
{
    if (!c->learned.ready) return fail(c, HHG_ESTATE, "no learned weights set");
    TRY(learned_scratch(c, l));
    Level &L = c->lv[l];
    for (int s = 0; s < sweeps; ++s) {
        TRY(residual_t<float>(c, l, f, u, L.r32, nullptr, st));
        HIPCHK(c, launch_learned_step(view<float>(c, l), c->learned, L.r32, L.logk32, u, L.invd32,
                                      (float)c->learned.omega, st));
    }
    return HHG_OK;
}

}  // namespace

// ================================================================ C ABI// ================================================================ C ABI
extern "C" {

hhg_status hhg_create_macro(const double *vert_xyz, int32_t n_vert, const int32_t *tet_vert,
                            int32_t n_tet, int32_t max_level, uint32_t flags, void *hip_stream,
                            hhg_ctx *out)
{
    if (out) *out = nullptr;
    if (!vert_xyz || !tet_vert || !out || n_vert <= 0 || n_tet <= 0 || n_tet >= (1 << 16))
        return fail(nullptr, HHG_EINVAL, "invalid mesh arguments");
    if (max_level < 0 || max_level > 10) return fail(nullptr, HHG_EINVAL, "max_level must be in [0, 10]");
    if (flags & ~(HHG_FLAG_NO_MODIFICATION | HHG_FLAG_COARSE_K_GEOMETRIC))
        return fail(nullptr, HHG_EINVAL, "unknown flag bits");
    for (int i = 0; i < 4 * n_tet; ++i)
        if (tet_vert[i] < 0 || tet_vert[i] >= n_vert) return fail(nullptr, HHG_EINVAL, "vertex id out of range");
    hhg_ctx c = new hhg_ctx_s();
    c->flags = flags;
    c->stream = (hipStream_t)hip_stream;
    c->max_level = max_level;
    Topology &tp = c->topo;
    tp.nv = n_vert;
    tp.nt = n_tet;
    tp.X.assign(vert_xyz, vert_xyz + 3 * n_vert);
    tp.tet.assign(tet_vert, tet_vert + 4 * n_tet);
    tp.vpos.assign(n_vert, -1);
    for (int i = 0; i < 4 * n_tet; ++i) tp.vpos[tet_vert[i]] = 1;
    for (int v = 0; v < n_vert; ++v)
        if (tp.vpos[v] == 1) tp.vpos[v] = tp.nvu++;
    std::vector<std::array<int, 2>> E;
    std::vector<std::array<int, 3>> F;
    for (int t = 0; t < n_tet; ++t) {
        const int *v = tet_vert + 4 * t;
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b) {
                if (v[a] == v[b]) { delete c; return fail(nullptr, HHG_EMESH, "tet %d repeats a vertex", t); }
                E.push_back({std::min(v[a], v[b]), std::max(v[a], v[b])});
            }
        for (int skip = 0; skip < 4; ++skip) {
            std::array<int, 3> f;
            int q = 0;
            for (int a = 0; a < 4; ++a)
                if (a != skip) f[q++] = v[a];
            std::sort(f.begin(), f.end());
            F.push_back(f);
        }
    }
    std::sort(E.begin(), E.end());
    std::sort(F.begin(), F.end());
    for (size_t i = 0; i < E.size(); ++i)
        if (i == 0 || E[i] != E[i - 1]) { tp.edges.push_back(E[i]); tp.e_val.push_back(0); }
        else {}
    for (size_t i = 0; i < F.size(); ++i) {
        if (i == 0 || F[i] != F[i - 1]) { tp.faces.push_back(F[i]); tp.f_val.push_back(0); }
        tp.f_val.back()++;
    }
    for (size_t f = 0; f < tp.faces.size(); ++f)
        if (tp.f_val[f] > 2) { delete c; return fail(nullptr, HHG_EMESH, "a face is shared by more than two tets"); }
    tp.v_val.assign(n_vert, 0);
    for (int t = 0; t < n_tet; ++t) {
        const int *v = tet_vert + 4 * t;
        for (int a = 0; a < 4; ++a) tp.v_val[v[a]]++;
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b) tp.e_val[tp.find_edge(v[a], v[b])]++;
    }
    tp.v_bnd.assign(n_vert, 0);
    tp.e_bnd.assign(tp.edges.size(), 0);
    tp.f_bnd.assign(tp.faces.size(), 0);
    for (size_t f = 0; f < tp.faces.size(); ++f) {
        if (tp.f_val[f] != 1) continue;
        tp.f_bnd[f] = 1;
        const auto &fv = tp.faces[f];
        for (int a = 0; a < 3; ++a) {
            tp.v_bnd[fv[a]] = 1;
            for (int b = a + 1; b < 3; ++b) tp.e_bnd[tp.find_edge(fv[a], fv[b])] = 1;
        }
    }
    // every tet must have positive volume
    for (int t = 0; t < n_tet; ++t) {
        double E0[NTYPE][4][4];
        if (!type_matrices(tp, t, 1, E0)) { delete c; return fail(nullptr, HHG_EMESH, "tet %d is degenerate", t); }
    }
    {
        const std::string why = conformity_error(tp.X, tp.tet, tp.nv, tp.nt, tp.edges, tp.faces, tp.f_val);
        if (!why.empty()) { delete c; return fail(nullptr, HHG_EMESH, "non-conforming macro mesh: %s", why.c_str()); }
    }
    c->lv.resize(max_level + 1);
    hhg_status s = HHG_OK;
    for (int l = 0; l <= max_level && s == HHG_OK; ++l) s = build_level(c, l);
    if (s == HHG_OK) {
        int64_t pc = 1024;
        for (int l = 0; l <= max_level; ++l) {
            Level &L = c->lv[l];
            const int64_t bp2 = (L.n_bnd + BLOCK - 1) / BLOCK;
            const int64_t gm = std::max({(int64_t)tp.nt * ((L.n_items + 3) / 4 + bp2),
                                         (int64_t)tp.nt * ((L.n_items2 + 3) / 4 + bp2),
                                         (int64_t)tp.nt * ((L.n_items2f + 3) / 4 + bp2),
                                         (int64_t)tp.nt * (L.n_items2 + (L.n_bnd + 63) / 64),
                                         (int64_t)tp.nt * (L.n_items2f + (L.n_bnd + 63) / 64),
                                         (int64_t)tp.nt * (L.n_itemsL + (L.n_bnd + 511) / 512)});
            const int64_t gv = (std::max((int64_t)tp.nt * L.bpt, gm) + 7) / 8 * 8;
            L.partial_bound = gv + (L.n_shared + BLOCK - 1) / BLOCK + (L.n_slots + BLOCK - 1) / BLOCK + 8;
            pc = std::max(pc, L.partial_bound);
        }
        c->partial_cap = pc;
        s = dalloc(c, &c->partial, pc);
        if (s == HHG_OK) s = dalloc(c, &c->dscalar, 16);
        if (s == HHG_OK) s = dalloc(c, &c->dflag, 4);
        if (s == HHG_OK && hipHostMalloc((void **)&c->hscalar, 16 * sizeof(double)) != hipSuccess)
            s = fail(c, HHG_ENOMEM, "hipHostMalloc failed");
    }
    if (s != HHG_OK) {
        g_create_error = c->err;
        hhg_destroy(c);
        return s;
    }
    c->coarse = default_coarse(c);
    {
        hipError_t e = hipSuccess;
        c->noalloc_scratch = noalloc_scratch_address(&e);
        if (!c->noalloc_scratch) {
            const hhg_status st = fail(c, HHG_EHIP, "scratch symbol lookup failed: %s", hipGetErrorString(e));
            g_create_error = c->err;
            hhg_destroy(c);
            return st;
        }
    }
    *out = c;
    return HHG_OK;
}

hhg_status hhg_destroy(hhg_ctx c)
{
    if (!c) return HHG_OK;
    (void)hipDeviceSynchronize();
    clear_graphs(c);
    for (hipEvent_t e : c->gev)
        if (e) (void)hipEventDestroy(e);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    for (void *p : c->allocs) (void)hipFree(p);
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    if (c->hscalar) (void)hipHostFree(c->hscalar);
    delete c;
    return HHG_OK;
}

const char *hhg_last_error(hhg_ctx c) { return c ? c->err.c_str() : g_create_error.c_str(); }

static hhg_status check_level(hhg_ctx c, int32_t level)
{
    if (!c) return HHG_EINVAL;
    if (level < 0 || level > c->max_level) return fail(c, HHG_EINVAL, "level %d out of range", level);
    return HHG_OK;
}

hhg_status hhg_vector_size(hhg_ctx c, int32_t level, int64_t *n_slots, int64_t *n_unknowns,
                           int64_t *n_nodes)
{
    TRY(check_level(c, level));
    const Level &L = c->lv[level];
    if (n_slots) *n_slots = L.n_slots;
    if (n_unknowns) *n_unknowns = L.n_unknowns;
    if (n_nodes) *n_nodes = L.n_nodes;
    return HHG_OK;
}

hhg_status hhg_node_coords(hhg_ctx c, int32_t level, double *xyz, uint8_t *dirichlet)
{
    TRY(check_level(c, level));
    if (!xyz) return fail(c, HHG_EINVAL, "xyz is NULL");
    const Level &L = c->lv[level];
    const Topology &tp = c->topo;
    for (int t = 0; t < tp.nt; ++t)
        for (int k = 0; k <= L.n; ++k)
            for (int j = 0; j + k <= L.n; ++j)
                for (int i = 0; i + j + k <= L.n; ++i) {
                    const int64_t ci = canon_index(tp, t, L.n, i, j, k, L.h_poff.data());
                    if (ci < 0 || ci >= L.n_nodes) return fail(c, HHG_EMESH, "canonical numbering out of range");
                    lattice_point(tp, t, L.n, i, j, k, xyz + 3 * ci);
                    if (dirichlet) dirichlet[ci] = (L.h_dmask[t] >> zero_pattern(L.n, i, j, k)) & 1;
                }
    return HHG_OK;
}

hhg_status hhg_to_canonical(hhg_ctx c, int32_t level, hhg_dtype dt, const void *v_slots, void *v_canon,
                            void *stream)
{
    TRY(check_level(c, level));
    if (!v_slots || !v_canon) return fail(c, HHG_EINVAL, "NULL vector");
    TRY(ensure_canon_maps(c, level));
    const Level &L = c->lv[level];
    hipStream_t st = pick(c, stream);
    if (dt == HHG_F64)
        HIPCHK(c, launch_to_canonical<double>((const double *)v_slots, L.canon2slot, (double *)v_canon, L.n_nodes, st));
    else if (dt == HHG_F32)
        HIPCHK(c, launch_to_canonical<float>((const float *)v_slots, L.canon2slot, (float *)v_canon, L.n_nodes, st));
    else return fail(c, HHG_EINVAL, "bad dtype");
    return HHG_OK;
}

hhg_status hhg_from_canonical(hhg_ctx c, int32_t level, hhg_dtype dt, const void *v_canon,
                              void *v_slots, void *stream)
{
    TRY(check_level(c, level));
    if (!v_slots || !v_canon) return fail(c, HHG_EINVAL, "NULL vector");
    TRY(ensure_canon_maps(c, level));
    const Level &L = c->lv[level];
    hipStream_t st = pick(c, stream);
    if (dt == HHG_F64)
        HIPCHK(c, launch_from_canonical<double>((const double *)v_canon, L.slot2canon, (double *)v_slots, L.n_slots, 0, L.S, L.Spad, st));
    else if (dt == HHG_F32)
        HIPCHK(c, launch_from_canonical<float>((const float *)v_canon, L.slot2canon, (float *)v_slots, L.n_slots, 0, L.S, L.Spad, st));
    else return fail(c, HHG_EINVAL, "bad dtype");
    return HHG_OK;
}

hhg_status hhg_set_coefficient(hhg_ctx c, const double *k, int on_device, void *stream)
{
    if (!c || !k) return fail(c, HHG_EINVAL, "NULL argument");
    hipStream_t st = pick(c, stream);
    const int Lmax = c->max_level;
    Level &F = c->lv[Lmax];
    TRY(ensure_canon_maps(c, Lmax));
    double *dk = nullptr;
    TRY(dalloc(c, &dk, F.n_nodes));
    auto release = [&]() { dfree(c, dk); };
    HIPCHK(c, hipMemcpyAsync(dk, k, F.n_nodes * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemsetAsync(c->dflag, 0, 4, st));
    HIPCHK(c, launch_positive_check(dk, F.n_nodes, c->dflag, st));
    int bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->dflag, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (bad) { release(); return fail(c, HHG_ECOEF, "coefficient must be positive and finite at every node"); }
    // Dirichlet slots also need k (rows next to the boundary read it): fill
    // every slot from its node, Dirichlet ones included; padding slots get 1
    HIPCHK(c, launch_fill<double>(F.k64, 1.0, F.n_slots, st));
    HIPCHK(c, launch_from_canonical<double>(dk, F.slot2canon, F.k64, F.n_slots, 1, F.S, F.Spad, st));
    HIPCHK(c, hipStreamSynchronize(st));
    release();
    for (int l = Lmax - 1; l >= 0; --l) {
        Level &Lc = c->lv[l], &Lf = c->lv[l + 1];
        HIPCHK(c, launch_fill<double>(Lc.k64, 1.0, Lc.n_slots, st));
        if (c->flags & HHG_FLAG_COARSE_K_GEOMETRIC) {
            TRY(build_coarsen_lists(c, l));
            HIPCHK(c, launch_coarsen(Lf.k64, Lf.n, Lc.k64, Lc.n, c->topo.nt, Lf.Spad, Lc.Spad, Lc.cg_n, Lc.cg_off,
                                     Lc.cg_fslot, Lc.cg_w, Lc.cg_coff, Lc.cg_cslot, st));
        } else {
            HIPCHK(c, launch_inject<double>(Lf.k64, Lf.n, Lc.k64, Lc.n, c->topo.nt, Lf.Spad, Lc.Spad, st));
        }
    }
    for (int l = 0; l <= Lmax; ++l) {
        Level &L = c->lv[l];
        HIPCHK(c, launch_convert<double, float>(L.k64, L.k32, L.n_slots, st));
        HIPCHK(c, launch_logk(L.k64, L.logk32, L.n_slots, st));
        if (L.n_shared > 0) {
            const int64_t ne = (int64_t)L.sh_w * L.n_shared;
            HIPCHK(c, launch_shared_coef(view<double>(c, l), L.sh_map, L.sh_cs64, L.sh_cn64, st));
            HIPCHK(c, launch_shared_coef_scaled(view<double>(c, l), L.sh_maps, L.sh_css64, st));
            HIPCHK(c, launch_convert<double, float>(L.sh_css64, L.sh_css32, (int64_t)L.sh_ws * L.n_shared, st));
            HIPCHK(c, launch_convert<double, float>(L.sh_cs64, L.sh_cs32, ne, st));
            HIPCHK(c, launch_convert<double, float>(L.sh_cn64, L.sh_cn32, ne, st));
        }
    }
    HIPCHK(c, hipStreamSynchronize(st));
    for (int l = 0; l <= Lmax; ++l) {
        TRY(build_modification(c, l));
        TRY(build_diag(c, l, st));
        Level &L = c->lv[l];
        if (L.st64) {
            HIPCHK(c, launch_store_stencils<double>(view<double>(c, l), L.st64, st));
            HIPCHK(c, launch_store_stencils<float>(view<double>(c, l), L.st32, st));
        }
    }
    c->have_k = true;
    c->oready[2] = c->oready[3] = false;  // the nodal and mixed solvers depend on k
    ++c->graph_epoch;
    TRY(build_coarse(c, st));
    return HHG_OK;
}

hhg_status hhg_set_coarse_level(hhg_ctx c, int32_t level)
{
    TRY(check_level(c, level));
    if (c->lv[level].n_unknowns < 1) return fail(c, HHG_EINVAL, "level %d has no unknowns", level);
    c->coarse = level;
    ++c->graph_epoch;
    if (c->have_k) TRY(build_coarse(c, c->stream));
    return HHG_OK;
}

hhg_status hhg_level_info(hhg_ctx c, int32_t level, double *lambda_max, int64_t *n_mod, int32_t *coarse)
{
    TRY(check_level(c, level));
    if (lambda_max) *lambda_max = c->lv[level].lam;
    if (n_mod) *n_mod = c->lv[level].n_corr;
    if (coarse) *coarse = c->coarse;
    return HHG_OK;
}

#define NEED_K(c)                                                                   \
    do {                                                                            \
        if (!(c)->have_k) return fail((c), HHG_ESTATE, "no coefficient set");       \
    } while (0)

hhg_status hhg_apply_scaled(hhg_ctx c, int32_t level, hhg_dtype dt, const void *u, void *y, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (!u || !y || u == y) return fail(c, HHG_EINVAL, "u and y must be distinct non-NULL vectors");
    hipStream_t st = pick(c, stream);
    if (dt == HHG_F64) return apply_scaled_t<double>(c, level, (const double *)u, (double *)y, st);
    if (dt == HHG_F32) return apply_scaled_t<float>(c, level, (const float *)u, (float *)y, st);
    return fail(c, HHG_EINVAL, "bad dtype");
}

hhg_status hhg_set_kernel_variant(int32_t variant)
{
    return set_march_variant(variant) == 0 ? HHG_OK : HHG_EINVAL;
}

hhg_status hhg_set_graphs(hhg_ctx c, int32_t enable)
{
    if (!c) return HHG_EINVAL;
    c->graphs = enable != 0;
    return HHG_OK;
}

hhg_status hhg_set_timing(hhg_ctx c, int32_t enable)
{
    if (!c) return HHG_EINVAL;
    c->timing = enable != 0;
    c->tev_used = 0;
    return HHG_OK;
}

hhg_status hhg_read_timing(hhg_ctx c, double *ms_total, int64_t *launches)
{
    if (!c || !ms_total || !launches) return HHG_EINVAL;
    double tot = 0.0;
    for (size_t q = 0; q < c->tev_used; ++q) {
        HIPCHK(c, hipEventSynchronize(c->tev[2 * q + 1]));
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->tev[2 * q], c->tev[2 * q + 1]));
        tot += ms;
    }
    *ms_total = tot;
    *launches = (int64_t)c->tev_used;
    c->tev_used = 0;
    return HHG_OK;
}

hhg_status hhg_apply_nodal(hhg_ctx c, int32_t level, hhg_dtype dt, const void *u, void *y, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (!u || !y || u == y) return fail(c, HHG_EINVAL, "u and y must be distinct non-NULL vectors");
    hipStream_t st = pick(c, stream);
    if (dt == HHG_F64) HIPCHK(c, launch_nodal<double>(view<double>(c, level), (const double *)u, (double *)y, st));
    else if (dt == HHG_F32) HIPCHK(c, launch_nodal<float>(view<float>(c, level), (const float *)u, (float *)y, st));
    else return fail(c, HHG_EINVAL, "bad dtype");
    return HHG_OK;
}

hhg_status hhg_set_tensor_coefficient(hhg_ctx c, const double *k6, int on_device, void *stream)
{
    if (!c || !k6) return fail(c, HHG_EINVAL, "NULL argument");
    hipStream_t st = pick(c, stream);
    const int Lmax = c->max_level;
    Level &F = c->lv[Lmax];
    TRY(ensure_canon_maps(c, Lmax));
    for (int l = 0; l <= Lmax; ++l) {
        Level &L = c->lv[l];
        if (!L.kt64) {
            TRY(dalloc(c, &L.kt64, 6 * L.n_slots));
            TRY(dalloc(c, &L.kt32, 6 * L.n_slots));
            TRY(dalloc(c, &L.kp64, NDIR / 2 * L.n_slots));
            TRY(dalloc(c, &L.kp32, NDIR / 2 * L.n_slots));
            const int64_t ne = (int64_t)L.sh_wt * L.n_shared;
            TRY(dalloc(c, &L.sh_ct64, ne));
            TRY(dalloc(c, &L.sh_ctn64, ne));
            TRY(dalloc(c, &L.sh_ct32, ne));
            TRY(dalloc(c, &L.sh_ctn32, ne));
        }
    }
    double *dk = nullptr;
    TRY(dalloc(c, &dk, 6 * F.n_nodes));
    HIPCHK(c, hipMemcpyAsync(dk, k6, 6 * F.n_nodes * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             st));
    for (int m = 0; m < 6; ++m) {
        // every slot from its node, Dirichlet ones included (rows next to the
        // boundary read them); padding slots 0
        double *km = F.kt64 + (int64_t)m * F.n_slots;
        HIPCHK(c, launch_fill<double>(km, 0.0, F.n_slots, st));
        HIPCHK(c, launch_from_canonical<double>(dk + (int64_t)m * F.n_nodes, F.slot2canon, km, F.n_slots, 1, F.S,
                                                F.Spad, st));
        for (int l = Lmax - 1; l >= 0; --l) {
            Level &Lc = c->lv[l], &Lf = c->lv[l + 1];
            double *kc = Lc.kt64 + (int64_t)m * Lc.n_slots;
            HIPCHK(c, launch_fill<double>(kc, 0.0, Lc.n_slots, st));
            HIPCHK(c, launch_inject<double>(Lf.kt64 + (int64_t)m * Lf.n_slots, Lf.n, kc, Lc.n, c->topo.nt, Lf.Spad,
                                            Lc.Spad, st));
        }
    }
    for (int l = 0; l <= Lmax; ++l) {
        Level &L = c->lv[l];
        HIPCHK(c, launch_convert<double, float>(L.kt64, L.kt32, 6 * L.n_slots, st));
        HIPCHK(c, launch_tensor_pairs(view<double>(c, l), L.kp64, st));
        HIPCHK(c, launch_convert<double, float>(L.kp64, L.kp32, NDIR / 2 * L.n_slots, st));
        if (L.n_shared > 0) {
            const int64_t ne = (int64_t)L.sh_wt * L.n_shared;
            HIPCHK(c, launch_tensor_shared_coef(view<double>(c, l), L.sh_mapt, L.sh_ct64, L.sh_ctn64, st));
            HIPCHK(c, launch_convert<double, float>(L.sh_ct64, L.sh_ct32, ne, st));
            HIPCHK(c, launch_convert<double, float>(L.sh_ctn64, L.sh_ctn32, ne, st));
        }
    }
    HIPCHK(c, hipStreamSynchronize(st));
    dfree(c, dk);
    c->have_tk = true;
    c->oready[0] = c->oready[1] = false;
    ++c->graph_epoch;
    return HHG_OK;
}

hhg_status hhg_apply_tensor(hhg_ctx c, int32_t level, hhg_dtype dt, const void *u, void *y, void *stream)
{
    TRY(check_level(c, level));
    if (!c->have_tk) return fail(c, HHG_ESTATE, "no tensor coefficient set");
    if (!u || !y || u == y) return fail(c, HHG_EINVAL, "u and y must be distinct non-NULL vectors");
    hipStream_t st = pick(c, stream);
    if (dt == HHG_F64)
        HIPCHK(c, launch_tensor<double>(view<double>(c, level), 0, MODE_APPLY, (const double *)u, nullptr, (double *)y,
                                        nullptr, nullptr, st));
    else if (dt == HHG_F32)
        HIPCHK(c, launch_tensor<float>(view<float>(c, level), 0, MODE_APPLY, (const float *)u, nullptr, (float *)y,
                                       nullptr, nullptr, st));
    else return fail(c, HHG_EINVAL, "bad dtype");
    return HHG_OK;
}

hhg_status hhg_apply_tensor_nodal(hhg_ctx c, int32_t level, hhg_dtype dt, const void *u, void *y, void *stream)
{
    TRY(check_level(c, level));
    if (!c->have_tk) return fail(c, HHG_ESTATE, "no tensor coefficient set");
    if (!u || !y || u == y) return fail(c, HHG_EINVAL, "u and y must be distinct non-NULL vectors");
    hipStream_t st = pick(c, stream);
    if (dt == HHG_F64)
        HIPCHK(c, launch_tensor<double>(view<double>(c, level), 1, MODE_APPLY, (const double *)u, nullptr, (double *)y,
                                        nullptr, nullptr, st));
    else if (dt == HHG_F32)
        HIPCHK(c, launch_tensor<float>(view<float>(c, level), 1, MODE_APPLY, (const float *)u, nullptr, (float *)y,
                                       nullptr, nullptr, st));
    else return fail(c, HHG_EINVAL, "bad dtype");
    return HHG_OK;
}

hhg_status hhg_store_stencils(hhg_ctx c, int32_t level)
{
    TRY(check_level(c, level));
    NEED_K(c);
    Level &L = c->lv[level];
    hipStream_t st = c->stream;
    if (!L.st64) {
        TRY(dalloc(c, &L.st64, (int64_t)15 * L.n_slots));
        hhg_status s = dalloc(c, &L.st32, (int64_t)15 * L.n_slots);
        if (s != HHG_OK) {
            dfree(c, L.st64);
            L.st64 = nullptr;
            return s;
        }
    }
    HIPCHK(c, launch_store_stencils<double>(view<double>(c, level), L.st64, st));
    HIPCHK(c, launch_store_stencils<float>(view<double>(c, level), L.st32, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return HHG_OK;
}

hhg_status hhg_apply_stored(hhg_ctx c, int32_t level, hhg_dtype dt, const void *u, void *y, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (!u || !y || u == y) return fail(c, HHG_EINVAL, "u and y must be distinct non-NULL vectors");
    const Level &L = c->lv[level];
    if (!L.st64) return fail(c, HHG_EINVAL, "stencils of level %d are not stored (hhg_store_stencils)", level);
    hipStream_t st = pick(c, stream);
    if (dt == HHG_F64)
        HIPCHK(c, launch_stored<double>(view<double>(c, level), corr<double>(c, level), L.st64, (const double *)u,
                                        (double *)y, st));
    else if (dt == HHG_F32)
        HIPCHK(c, launch_stored<float>(view<float>(c, level), corr<float>(c, level), L.st32, (const float *)u,
                                       (float *)y, st));
    else return fail(c, HHG_EINVAL, "bad dtype");
    return HHG_OK;
}

hhg_status hhg_apply_mixed(hhg_ctx c, int32_t level, hhg_dtype dt, int32_t nodal_primitives, const void *u,
                           void *y, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (!u || !y || u == y) return fail(c, HHG_EINVAL, "u and y must be distinct non-NULL vectors");
    if (nodal_primitives < 0 || nodal_primitives > 7) return fail(c, HHG_EINVAL, "nodal_primitives must be in 0..7");
    hipStream_t st = pick(c, stream);
    if (dt == HHG_F64)
        HIPCHK(c, launch_mixed<double>(view<double>(c, level), corr<double>(c, level), (const double *)u, (double *)y,
                                       nodal_primitives, st));
    else if (dt == HHG_F32)
        HIPCHK(c, launch_mixed<float>(view<float>(c, level), corr<float>(c, level), (const float *)u, (float *)y,
                                      nodal_primitives, st));
    else return fail(c, HHG_EINVAL, "bad dtype");
    return HHG_OK;
}

hhg_status hhg_residual(hhg_ctx c, int32_t level, hhg_dtype dt, const void *f, const void *u, void *r,
                        double *norm2_out, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (!f || !u || !r || r == u || r == f) return fail(c, HHG_EINVAL, "bad vectors");
    hipStream_t st = pick(c, stream);
    if (dt == HHG_F64) return residual_t<double>(c, level, (const double *)f, (const double *)u, (double *)r, norm2_out, st);
    if (dt == HHG_F32) return residual_t<float>(c, level, (const float *)f, (const float *)u, (float *)r, norm2_out, st);
    return fail(c, HHG_EINVAL, "bad dtype");
}

hhg_status hhg_residual_noalloc(hhg_ctx c, int32_t level, hhg_dtype dt, const void *f, const void *u, void *r,
                                double *norm2_out, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (!f || !u || !r || r == u || r == f) return fail(c, HHG_EINVAL, "bad vectors");
    if (dt != HHG_F64 && dt != HHG_F32) return fail(c, HHG_EINVAL, "bad dtype");
    if (!c->noalloc_scratch) return fail(c, HHG_ESTATE, "no scratch address for this context's device");
    const int64_t need = NOALLOC_PARTIAL_AT + c->lv[level].partial_bound;
    if (need > NOALLOC_SCRATCH_DOUBLES)
        return fail(c, HHG_EINVAL,
                    "level %d needs %lld scratch values for its residual norm; the static scratch holds %lld",
                    level, (long long)need, (long long)NOALLOC_SCRATCH_DOUBLES);
    hipStream_t st = pick(c, stream);
    // every block partial the reduction reads is written by this call's
    // kernels first, so nothing in the scratch needs clearing
    double *const partial = c->noalloc_scratch + NOALLOC_PARTIAL_AT;
    double *const value = c->noalloc_scratch;
    if (dt == HHG_F64)
        return residual_t<double>(c, level, (const double *)f, (const double *)u, (double *)r, norm2_out, st,
                                  partial, value);
    return residual_t<float>(c, level, (const float *)f, (const float *)u, (float *)r, norm2_out, st, partial,
                             value);
}

hhg_status hhg_smooth(hhg_ctx c, int32_t level, hhg_dtype dt, hhg_smoother sm, int32_t sweeps, double omega,
                      const void *f, void *u, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (!f || !u || f == u || sweeps < 0) return fail(c, HHG_EINVAL, "bad arguments");
    hipStream_t st = pick(c, stream);
    if (sm == HHG_LEARNED) {
        if (dt == HHG_F64) return learned_smooth_t<double>(c, level, sweeps, (const double *)f, (double *)u, st);
        if (dt == HHG_F32) return learned_smooth_t<float>(c, level, sweeps, (const float *)f, (float *)u, st);
        return fail(c, HHG_EINVAL, "bad dtype");
    }
    if (sm != HHG_JACOBI && sm != HHG_CHEBYSHEV) return fail(c, HHG_EINVAL, "bad smoother");
    if (dt == HHG_F64) return smooth_t<double>(c, level, sm, sweeps, omega, (const double *)f, (double *)u, st);
    if (dt == HHG_F32) return smooth_t<float>(c, level, sm, sweeps, omega, (const float *)f, (float *)u, st);
    return fail(c, HHG_EINVAL, "bad dtype");
}

hhg_status hhg_vcycle(hhg_ctx c, int32_t level, hhg_dtype dt, int32_t pre, int32_t post, hhg_smoother sm,
                      const void *f, void *u, double *rel_res_out, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (!f || !u || f == u || pre < 0 || post < 0) return fail(c, HHG_EINVAL, "bad arguments");
    if (level < c->coarse) return fail(c, HHG_EINVAL, "level below the coarse level");
    if (sm != HHG_JACOBI && sm != HHG_CHEBYSHEV && sm != HHG_LEARNED) return fail(c, HHG_EINVAL, "bad smoother");
    hipStream_t st = pick(c, stream);
    Level &L = c->lv[level];
    if (dt == HHG_F64) {
        TRY(vcycle_t<double>(c, level, (const double *)f, (double *)u, pre, post, sm, st));
        if (rel_res_out) {
            double nr, nf;
            TRY(residual_t<double>(c, level, (const double *)f, (const double *)u, L.r64, &nr, st));
            HIPCHK(c, launch_fill<double>(L.d64, 0.0, L.n_slots, st));
            TRY(residual_t<double>(c, level, (const double *)f, L.d64, L.r64, &nf, st));
            *rel_res_out = nf > 0 ? nr / nf : nr;
        }
        return HHG_OK;
    }
    if (dt == HHG_F32) {
        TRY(vcycle_t<float>(c, level, (const float *)f, (float *)u, pre, post, sm, st));
        if (rel_res_out) {
            double nr, nf;
            TRY(residual_t<float>(c, level, (const float *)f, (const float *)u, L.r32, &nr, st));
            HIPCHK(c, launch_fill<float>(L.d32, 0.0f, L.n_slots, st));
            TRY(residual_t<float>(c, level, (const float *)f, L.d32, L.r32, &nf, st));
            *rel_res_out = nf > 0 ? nr / nf : nr;
        }
        return HHG_OK;
    }
    return fail(c, HHG_EINVAL, "bad dtype");
}

namespace {
// the solve loop of hhg_solve / hhg_solve_tensor on the operator c->op
hhg_status solve_impl(hhg_ctx c, int32_t level, hhg_solve_mode mode, int32_t pre, int32_t post, double tol,
                      int32_t max_iter, const double *f, double *u, hhg_solve_stats *stats, void *stream)
{
    if (!f || !u || f == u || max_iter < 0 || pre < 0 || post < 0) return fail(c, HHG_EINVAL, "bad arguments");
    if (level < c->coarse) return fail(c, HHG_EINVAL, "level below the coarse level");
    if (mode != HHG_SOLVE_F64 && mode != HHG_SOLVE_MIXED && mode != HHG_SOLVE_LEARNED)
        return fail(c, HHG_EINVAL, "bad solve mode");
    hipStream_t st = pick(c, stream);
    Level &L = c->lv[level];
    HIPCHK(c, hipStreamSynchronize(st));
    const auto t0 = std::chrono::steady_clock::now();
    double nf = 0.0, nr = 0.0;
    // |f| over the unknowns: residual of the zero vector
    HIPCHK(c, launch_fill<double>(L.d64, 0.0, L.n_slots, st));
    TRY(residual_t<double>(c, level, f, L.d64, L.r64, &nf, st));
    if (!(nf > 0.0)) nf = 1.0;
    std::vector<double> hist;
    std::vector<int> cyc;  // V-cycles done before each entry of hist
    int cycles = 0;
    // FP32 V-cycles per refinement step: two in the plain mixed mode (the FP64
    // residual, its conversion and the correction's update then run once per
    // two cycles); one with the learned smoother, whose fallback judges each
    // cycle's contraction
    const int inner = mode == HHG_SOLVE_MIXED ? 2 : 1;
    int fallback = 0;
    bool use_learned = mode == HHG_SOLVE_LEARNED;
    const LearnedState &LS = c->learned;
    // the plain cycle's contraction, measured once from the same iterate as
    // a learned cycle (cycle LEARNED_PROBE_CYCLE), when a margin is set
    const bool probe = use_learned && LS.plain_margin > 0.0;
    double q_plain = -1.0;
    bool probe_pending = false;  // the last cycle was the probe's learned one
    if (use_learned && !L.ubak) TRY(dalloc(c, &L.ubak, L.n_slots));
    if (probe && !L.uprobe) TRY(dalloc(c, &L.uprobe, L.n_slots));
    for (int it = 0;; ++it) {
        TRY(residual_t<double>(c, level, f, u, L.r64, &nr, st));
        hist.push_back(nr / nf);
        cyc.push_back(cycles);
        // fallback: a learned cycle must keep the residual finite, contract
        // at least by the accepted rate and, once the plain cycle's
        // contraction is known, by no less than margin x that contraction;
        // otherwise its result is replaced (by the probe's plain result after
        // the probe, else by the iterate before the cycle) and the solve
        // continues with Chebyshev smoothing
        if (use_learned && it >= 1) {
            const double q = hist[it] / hist[it - 1];
            double bound = LS.fallback_rate;
            if (q_plain > 0.0) bound = std::min(bound, LS.plain_margin * q_plain);
            if (!std::isfinite(nr) || !(q <= bound)) {
                use_learned = false;
                fallback = 1;
                HIPCHK(c, hipMemcpyAsync(u, probe_pending ? L.uprobe : L.ubak, L.n_slots * sizeof(double),
                                         hipMemcpyDeviceToDevice, st));
                TRY(residual_t<double>(c, level, f, u, L.r64, &nr, st));
                hist.back() = nr / nf;
            }
        }
        probe_pending = false;
        if (!std::isfinite(nr)) break;
        if (hist.back() <= tol || cycles >= max_iter) break;
        if (mode == HHG_SOLVE_F64) {
            TRY(vcycle_run<double>(c, level, f, u, pre, post, HHG_CHEBYSHEV, st));
            ++cycles;
        } else {
            HIPCHK(c, launch_convert<double, float>(L.r64, L.f32, L.n_slots, st));
            if (use_learned && probe && it == LEARNED_PROBE_CYCLE) {
                // the plain cycle from this iterate, into uprobe
                HIPCHK(c, launch_fill<float>(L.u32, 0.0f, L.n_slots, st));
                TRY(vcycle_run<float>(c, level, L.f32, L.u32, pre, post, HHG_CHEBYSHEV, st));
                HIPCHK(c, hipMemcpyAsync(L.uprobe, u, L.n_slots * sizeof(double), hipMemcpyDeviceToDevice, st));
                HIPCHK(c, launch_add_f32_to_f64(L.uprobe, L.u32, L.n_slots, st));
            }
            if (use_learned)
                HIPCHK(c, hipMemcpyAsync(L.ubak, u, L.n_slots * sizeof(double), hipMemcpyDeviceToDevice, st));
            HIPCHK(c, launch_fill<float>(L.u32, 0.0f, L.n_slots, st));
            for (int m = 0; m < inner && cycles < max_iter; ++m, ++cycles)
                TRY(vcycle_run<float>(c, level, L.f32, L.u32, pre, post, use_learned ? HHG_LEARNED : HHG_CHEBYSHEV,
                                      st));
            HIPCHK(c, launch_add_f32_to_f64(u, L.u32, L.n_slots, st));
            if (use_learned && probe && it == LEARNED_PROBE_CYCLE) {
                double np = 0.0;
                TRY(residual_t<double>(c, level, f, L.uprobe, L.r64, &np, st));
                q_plain = (np / nf) / hist[it];
                probe_pending = true;
            }
        }
    }
    HIPCHK(c, hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) {
        // rho per V-cycle, from the first residual after five cycles (else
        // the initial one) to the last
        const int n = (int)hist.size() - 1;
        int j = 0;
        while (j < n && cyc[j] < 5) ++j;
        if (cyc[n] - cyc[j] <= 0) j = 0;
        stats->iterations = cycles;
        stats->fallback = fallback;
        stats->rel_residual = hist.back();
        stats->seconds = secs;
        stats->rho = cyc[n] > cyc[j] ? std::pow(hist[n] / hist[j], 1.0 / (cyc[n] - cyc[j])) : 0.0;
    }
    return fallback ? HHG_WFALLBACK : HHG_OK;
}

// operator selection for the duration of a solve
struct OpScope {
    hhg_ctx c;
    OpScope(hhg_ctx c_, int op) : c(c_) { c->op = op; }
    ~OpScope() { c->op = 0; }
};

// inverse diagonals, Gershgorin bounds and the coarse inverse of operator op
// (1..4 as hhg_ctx_s::op; the mixed operator for c->mix_mask)
hhg_status ensure_op_solver(hhg_ctx c, int op)
{
    const int q = op - 1;
    if (c->oready[q] && c->oco_level[q] == c->coarse && (op != 4 || c->omask == c->mix_mask)) return HHG_OK;
    hipStream_t st = c->stream;
    // the levels a cycle visits (below the coarse level there may be no rows)
    for (int l = c->coarse; l <= c->max_level; ++l) {
        Level &L = c->lv[l];
        if (tensor_partial_count(L.n, c->topo.nt, L.n_shared) > c->partial_cap)
            return fail(c, HHG_EINVAL, "level %d: reduction buffer too small for the diagonal kernels", l);
        if (!L.oinvd64[q]) {
            TRY(dalloc(c, &L.oinvd64[q], L.n_slots));
            TRY(dalloc(c, &L.oinvd32[q], L.n_slots));
        }
        if (op == 4) {
            // the scaled operator's diagonal (with its modification) on every
            // row, the nodal one on the rows of the chosen primitives
            HIPCHK(c, hipMemcpyAsync(L.oinvd64[q], L.invd64, L.n_slots * 8, hipMemcpyDeviceToDevice, st));
            HIPCHK(c, launch_invert_diag<double>(L.oinvd64[q], L.n_slots, st));
        } else {
            // slots without a row (Dirichlet, padding) keep 1: their residual is 0
            HIPCHK(c, launch_fill<double>(L.oinvd64[q], 1.0, L.n_slots, st));
        }
        // form q: 0 / 1 the tensor forms, 2 scalar nodal, 3 the mixed operator's nodal rows
        int np = 0;
        HIPCHK(c, launch_form_diag(view<double>(c, l), q, c->mix_mask, L.oinvd64[q], c->partial, &np, st));
        HIPCHK(c, launch_reduce(c->partial, np, 1, c->dscalar, st));
        HIPCHK(c, hipMemcpyAsync(c->hscalar, c->dscalar, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        L.olam[q] = op == 4 ? std::max(L.lam, c->hscalar[0]) : c->hscalar[0];
        if (!(L.olam[q] > 0.0) || !std::isfinite(L.olam[q]))
            return fail(c, HHG_ECOEF, "level %d: operator %d has a non-positive diagonal", l, op);
        HIPCHK(c, launch_invert_diag<double>(L.oinvd64[q], L.n_slots, st));
        HIPCHK(c, launch_convert<double, float>(L.oinvd64[q], L.oinvd32[q], L.n_slots, st));
    }
    TRY(build_coarse(c, st, op));
    ++c->graph_epoch;
    c->oco_level[q] = c->coarse;
    if (op == 4) c->omask = c->mix_mask;
    c->oready[q] = true;
    return HHG_OK;
}
}  // namespace

hhg_status hhg_solve(hhg_ctx c, int32_t level, hhg_solve_mode mode, int32_t pre, int32_t post, double tol,
                     int32_t max_iter, const double *f, double *u, hhg_solve_stats *stats, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (mode == HHG_SOLVE_LEARNED && !c->learned.ready) return fail(c, HHG_ESTATE, "no learned weights set");
    return solve_impl(c, level, mode, pre, post, tol, max_iter, f, u, stats, stream);
}

hhg_status hhg_solve_tensor(hhg_ctx c, int32_t level, int32_t form, hhg_solve_mode mode, int32_t pre, int32_t post,
                            double tol, int32_t max_iter, const double *f, double *u, hhg_solve_stats *stats,
                            void *stream)
{
    TRY(check_level(c, level));
    if (!c->have_tk) return fail(c, HHG_ESTATE, "no tensor coefficient set");
    if (form != 0 && form != 1) return fail(c, HHG_EINVAL, "form must be 0 (scaled) or 1 (nodal)");
    if (mode != HHG_SOLVE_F64 && mode != HHG_SOLVE_MIXED)
        return fail(c, HHG_EINVAL, "tensor solves take HHG_SOLVE_F64 or HHG_SOLVE_MIXED");
    TRY(ensure_op_solver(c, 1 + form));
    OpScope scope(c, 1 + form);
    return solve_impl(c, level, mode, pre, post, tol, max_iter, f, u, stats, stream);
}

hhg_status hhg_solve_form(hhg_ctx c, int32_t level, int32_t form, int32_t nodal_primitives, hhg_solve_mode mode,
                          int32_t pre, int32_t post, double tol, int32_t max_iter, const double *f, double *u,
                          hhg_solve_stats *stats, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (form == HHG_FORM_SCALED) {
        if (mode == HHG_SOLVE_LEARNED && !c->learned.ready) return fail(c, HHG_ESTATE, "no learned weights set");
        return solve_impl(c, level, mode, pre, post, tol, max_iter, f, u, stats, stream);
    }
    if (form != HHG_FORM_NODAL && form != HHG_FORM_MIXED) return fail(c, HHG_EINVAL, "bad form");
    if (form == HHG_FORM_MIXED && (nodal_primitives & ~7))
        return fail(c, HHG_EINVAL, "nodal_primitives must be a combination of 1, 2 and 4");
    if (mode != HHG_SOLVE_F64 && mode != HHG_SOLVE_MIXED)
        return fail(c, HHG_EINVAL, "nodal and mixed forms take HHG_SOLVE_F64 or HHG_SOLVE_MIXED");
    const int op = form == HHG_FORM_NODAL ? 3 : 4;
    c->mix_mask = form == HHG_FORM_MIXED ? nodal_primitives : 0;
    TRY(ensure_op_solver(c, op));
    OpScope scope(c, op);
    return solve_impl(c, level, mode, pre, post, tol, max_iter, f, u, stats, stream);
}

hhg_status hhg_learned_set_weights(hhg_ctx c, const float *w, int64_t n)
{
    if (!c || !w) return fail(c, HHG_EINVAL, "NULL argument");
    if (n != LN_NPARAM) return fail(c, HHG_EINVAL, "expected %d parameters, got %lld", LN_NPARAM, (long long)n);
    for (int64_t q = 0; q < n; ++q)
        if (!std::isfinite(w[q])) return fail(c, HHG_EINVAL, "non-finite weight %lld", (long long)q);
    LearnedState &S = c->learned;
    if (!S.w32) {
        TRY(dalloc(c, &S.w32, LN_NPARAM));
        TRY(dalloc(c, &S.wbf, LN_NPARAM));
        TRY(dalloc(c, &S.dgrad, LN_NPARAM));
    }
    HIPCHK(c, hipMemcpy(S.w32, w, LN_NPARAM * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(c, launch_weights_bf16(S.w32, S.wbf, LN_NPARAM, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    S.ready = true;
    return HHG_OK;
}

hhg_status hhg_learned_set_fallback(hhg_ctx c, double max_rate, double plain_margin)
{
    if (!c || !(max_rate > 0.0)) return fail(c, HHG_EINVAL, "fallback rate must be positive");
    if (!(plain_margin >= 0.0) || !std::isfinite(plain_margin))
        return fail(c, HHG_EINVAL, "plain-cycle margin must be finite and >= 0");
    c->learned.fallback_rate = max_rate;
    c->learned.plain_margin = plain_margin;
    return HHG_OK;
}

hhg_status hhg_learned_forward(hhg_ctx c, int32_t level, const float *r, float *c_out, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (!c->learned.ready) return fail(c, HHG_ESTATE, "no learned weights set");
    if (!r || !c_out || (const void *)r == (const void *)c_out) return fail(c, HHG_EINVAL, "bad vectors");
    Level &L = c->lv[level];
    HIPCHK(c, launch_learned_forward<float>(view<float>(c, level), c->learned, r, L.logk32, c_out,
                                            pick(c, stream)));
    return HHG_OK;
}

static hhg_status learned_grad_to_host(hhg_ctx c, int level, const float *r, const float *g, float *dw,
                                       hipStream_t st)
{
    LearnedState &S = c->learned;
    const int nb = learned_bwd_blocks(view<float>(c, level));
    if (nb > S.gpart_blocks) {
        if (S.gpart) dfree(c, S.gpart);
        TRY(dalloc(c, &S.gpart, (int64_t)nb * LN_NPARAM));
        S.gpart_blocks = nb;
    }
    HIPCHK(c, launch_learned_backward(view<float>(c, level), S, r, c->lv[level].logk32, g, st));
    HIPCHK(c, hipMemcpyAsync(dw, S.dgrad, LN_NPARAM * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    return HHG_OK;
}

hhg_status hhg_learned_backward(hhg_ctx c, int32_t level, const float *r, const float *g, float *dw,
                                void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (!c->learned.ready) return fail(c, HHG_ESTATE, "no learned weights set");
    if (!r || !g || !dw) return fail(c, HHG_EINVAL, "NULL argument");
    return learned_grad_to_host(c, level, r, g, dw, pick(c, stream));
}

hhg_status hhg_learned_loss_grad(hhg_ctx c, int32_t level, const float *r, const float *e, double *loss,
                                 float *dw, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (!c->learned.ready) return fail(c, HHG_ESTATE, "no learned weights set");
    if (!r || !e || !loss || !dw) return fail(c, HHG_EINVAL, "NULL argument");
    hipStream_t st = pick(c, stream);
    TRY(learned_scratch(c, level));
    TRY(ensure_own(c, level));
    Level &L = c->lv[level];
    float *sc = L.lt[0], *sv = L.lt[1], *e1 = L.lt[2], *ae1 = L.lt[3], *ae = L.lt[4], *g = L.lt[5];
    const float om = (float)c->learned.omega;
    HIPCHK(c, launch_learned_forward_full(view<float>(c, level), c->learned, r, L.logk32, nullptr, sc, sv, st));
    HIPCHK(c, launch_learned_err(e, r, sc, L.invd32, om, e1, L.n_slots, st));
    TRY(apply_scaled_t<float>(c, level, e1, ae1, st));
    TRY(apply_scaled_t<float>(c, level, e, ae, st));
    hhg_status err;
    const double e0 = dot_owned(c, level, e, ae, st, &err);
    if (err) return err;
    const double ee = dot_owned(c, level, e1, ae1, st, &err);
    if (err) return err;
    if (!(e0 > 0.0)) return fail(c, HHG_EINVAL, "training sample has zero energy");
    *loss = ee / e0;
    HIPCHK(c, launch_learned_lossgrad(ae1, sv, L.invd32, 1.0 / e0, g, L.n_slots, st));
    return learned_grad_to_host(c, level, r, g, dw, st);
}

hhg_status hhg_training_pair(hhg_ctx c, int32_t level, const double *f, const double *u, const double *us,
                             float *r_out, float *e_out, void *stream)
{
    TRY(check_level(c, level));
    NEED_K(c);
    if (!f || !u || !us || !r_out || !e_out) return fail(c, HHG_EINVAL, "NULL argument");
    hipStream_t st = pick(c, stream);
    Level &L = c->lv[level];
    TRY(residual_t<double>(c, level, f, u, L.r64, nullptr, st));
    HIPCHK(c, launch_pair(L.r64, us, u, r_out, e_out, L.n_slots, st));
    return HHG_OK;
}

hhg_status hhg_adam_update(float *w, float *m, float *v, const float *g, int64_t n, int32_t t, double lr,
                           double b1, double b2, double eps)
{
    if (!w || !m || !v || !g || n <= 0 || t < 1) return HHG_EINVAL;
    const double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
    for (int64_t q = 0; q < n; ++q) {
        m[q] = (float)(b1 * m[q] + (1.0 - b1) * g[q]);
        v[q] = (float)(b2 * v[q] + (1.0 - b2) * (double)g[q] * g[q]);
        const double mh = m[q] / c1, vh = v[q] / c2;
        w[q] = (float)(w[q] - lr * mh / (std::sqrt(vh) + eps));
    }
    return HHG_OK;
}

}  // extern "C"
