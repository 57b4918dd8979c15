// 2D variant: P1 on uniformly refined triangular macro meshes with stencil
// scaling and the exact pre-asymptotic modification of Sec. 4.1 (MA2), and
// nodal integration as the comparison (eq. (standardfe)).
//
// Layout.  Macro triangle T with vertices (v0, v1, v2) carries the lattice
// points (i, j), i + j <= n = 2^level, at (w0 X0 + w1 X1 + w2 X2) / n with
// weights w = (n-i-j, i, j); its slots are row-major in j:
// slot(i, j) = j (n+1) - j (j-1) / 2 + i, padded per triangle to Spad.  Nodes
// on macro edges and vertices have one copy per triangle holding them; all
// copies hold the same value.
//
// Operators.  Every fine element of T has T's element matrix A_T (up cells
// are scaled translates, down cells point reflections).  An interior lattice
// edge of direction d lies in two elements, so the scaled interior row is
//   y_a = sum_d A_T[pair(d)] (k_a + k_d) (u_d - u_a)
// (pair: (1,0) -> A[0,1], (0,1) -> A[0,2], (-1,1) -> A[1,2], and negatives),
// evaluated on the fly.  Rows of nodes on shared macro edges / vertices take
// merged coefficients built from the elements of every copy; MA2 changes the
// factor of gray edges (A_T entry > 0) where it triggers, through those
// merged rows and a per-row correction list for interior rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "hhg2d.h"

namespace {

constexpr int B2 = 256;

// lattice directions (di, dj): pairs d and d + 3 are opposite
constexpr int D2[6][2] = {{1, 0}, {0, 1}, {-1, 1}, {-1, 0}, {0, -1}, {1, -1}};
// element-matrix pair (local vertices) of each direction
constexpr int PAIR[6][2] = {{0, 1}, {0, 2}, {1, 2}, {0, 1}, {0, 2}, {1, 2}};
// the six elements around a node: vertex offsets (local vertices 0, 1, 2)
// and the node's local index
struct El { int off[3][2]; int me; };
constexpr El AROUND[6] = {
    {{{0, 0}, {1, 0}, {0, 1}}, 0},    // up cell (i, j)
    {{{-1, 0}, {0, 0}, {-1, 1}}, 1},  // up cell (i-1, j)
    {{{0, -1}, {1, -1}, {0, 0}}, 2},  // up cell (i, j-1)
    {{{0, 0}, {-1, 0}, {0, -1}}, 0},  // down cell (i-1, j-1): (i,j) is its vertex 0
    {{{1, 0}, {0, 0}, {1, -1}}, 1},   // down cell (i, j-1)
    {{{0, 1}, {-1, 1}, {0, 0}}, 2},   // down cell (i-1, j)
};

__host__ __device__ inline bool in_tri(int n, int i, int j) { return i >= 0 && j >= 0 && i + j <= n; }
__host__ __device__ inline int64_t slot_of(int n, int i, int j)
{
    return (int64_t)j * (n + 1) - (int64_t)j * (j - 1) / 2 + i;
}
__host__ __device__ constexpr int dir_of(int di, int dj)
{
    for (int d = 0; d < 6; ++d)
        if (D2[d][0] == di && D2[d][1] == dj) return d;
    return -1;
}

struct Shared {
    std::vector<int64_t> self;              // global slot of the first copy
    std::vector<int32_t> off;               // copies of row q: [off[q], off[q+1])
    std::vector<int64_t> cslot;             // global slot of every copy
    std::vector<std::vector<std::pair<int, int>>> copy;  // (triangle, slot) per copy, host
};

}  // namespace

struct hhg2d_ctx_s {
    int n = 0, nt = 0, level = 0;
    uint32_t flags = 0;
    int64_t S = 0, Spad = 0, n_slots = 0, n_nodes = 0, n_unknowns = 0;
    std::vector<double> X;                  // (nv, 2)
    std::vector<int> T;                     // (nt, 3)
    std::vector<double> A;                  // (nt, 3, 3) element matrices of the macro triangles
    std::vector<double> lam;                // lambda_min per macro triangle
    std::vector<int64_t> slot2canon;        // per global slot (padding -1)
    std::vector<int64_t> canon2slot;        // first copy of each node
    std::vector<double> node_xy;            // (n_nodes, 2)
    std::vector<uint8_t> dir_node;          // Dirichlet per node
    std::vector<int64_t> dir_slots;         // every Dirichlet copy
    Shared sh;                              // shared (macro edge / vertex) unknown rows
    std::vector<double> k_slot;             // k per global slot (host)
    bool have_k = false;
    int64_t n_mod = 0;
    // device
    double *w64 = nullptr; float *w32 = nullptr;      // (nt, 3) half-stencil weights A[pair]
    double *d_A = nullptr;                            // (nt, 9) element matrices (nodal rows)
    double *k64 = nullptr; float *k32 = nullptr;
    int64_t *d_s2c = nullptr, *d_c2s = nullptr, *d_dir = nullptr;
    // shared rows: CSR over entries (neighbour slot, coefficient); copies
    int n_sh = 0;
    int32_t *d_sh_eoff = nullptr, *d_sh_off = nullptr;
    int64_t *d_sh_self = nullptr, *d_sh_nb = nullptr, *d_sh_cslot = nullptr;
    double *d_sh_cs64 = nullptr, *d_sh_cn64 = nullptr;
    float *d_sh_cs32 = nullptr, *d_sh_cn32 = nullptr;
    // MA2 corrections of interior rows: row slot, two neighbour slots, deltas
    int64_t n_corr = 0;
    int64_t *d_c_row = nullptr, *d_c_nb = nullptr;
    double *d_c_dl64 = nullptr; float *d_c_dl32 = nullptr;
    std::vector<void *> allocs;
    std::string err;
};

namespace {

hhg_status fail2(hhg2d_ctx c, hhg_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}
#define TRY2(x)                                  \
    do {                                         \
        hhg_status s_ = (x);                     \
        if (s_ != HHG_OK) return s_;             \
    } while (0)
#define HIP2(c, x)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) return fail2(c, HHG_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
hhg_status dalloc2(hhg2d_ctx c, T **p, int64_t n)
{
    *p = nullptr;
    if (n <= 0) n = 1;
    void *q = nullptr;
    if (hipMalloc(&q, (size_t)n * sizeof(T)) != hipSuccess)
        return fail2(c, HHG_ENOMEM, "hipMalloc of %lld bytes failed", (long long)(n * sizeof(T)));
    c->allocs.push_back(q);
    *p = (T *)q;
    return HHG_OK;
}
template <typename T>
hhg_status upload2(hhg2d_ctx c, T **p, const std::vector<T> &h)
{
    if (!*p) TRY2(dalloc2(c, p, (int64_t)h.size()));
    if (!h.empty()) HIP2(c, hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return HHG_OK;
}

// element matrix |t| G G^T of a triangle; false if degenerate
bool element_matrix(const double P[3][2], double A[3][3])
{
    const double e1x = P[1][0] - P[0][0], e1y = P[1][1] - P[0][1];
    const double e2x = P[2][0] - P[0][0], e2y = P[2][1] - P[0][1];
    const double det = e1x * e2y - e1y * e2x;
    if (!(std::fabs(det) > 0)) return false;
    // gradients of the barycentric functions 1 and 2 (rows of J^{-1})
    const double g1[2] = {e2y / det, -e2x / det}, g2[2] = {-e1y / det, e1x / det};
    const double g0[2] = {-g1[0] - g2[0], -g1[1] - g2[1]};
    const double *g[3] = {g0, g1, g2};
    const double area = std::fabs(det) / 2;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A[a][b] = area * (g[a][0] * g[b][0] + g[a][1] * g[b][1]);
    return true;
}

// smallest non-degenerate eigenvalue of A x = lambda B x, B = 3I - 11^T: on
// the complement of the constants (orthonormal basis q1, q2) B is 3 I
double lambda_min_T(const double A[3][3])
{
    const double s2 = std::sqrt(2.0), s6 = std::sqrt(6.0);
    const double q[2][3] = {{1 / s2, -1 / s2, 0}, {1 / s6, 1 / s6, -2 / s6}};
    double R[2][2];
    for (int p = 0; p < 2; ++p)
        for (int r = 0; r < 2; ++r) {
            double v = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) v += q[p][a] * A[a][b] * q[r][b];
            R[p][r] = v;
        }
    const double tr = R[0][0] + R[1][1], dt = R[0][0] * R[1][1] - R[0][1] * R[1][0];
    const double disc = std::sqrt(std::max(0.0, tr * tr / 4 - dt));
    return (tr / 2 - disc) / 3.0;
}

// ---------------------------------------------------------------- kernels
// Interior rows by column marching: a wave owns 64 consecutive
// columns c = i0 - 1 + lane (lanes 1..62 produce rows, lanes 0 and 63 only
// feed their neighbours) and walks rows j0..j1 holding u and k of rows j-1,
// j, j+1 in registers; per row it loads row j+2 once (coalesced along the
// row) and takes the in-row and diagonal neighbours from the adjacent lanes.
// jc rows per wave: the launcher takes the largest of 64/32/16/8 that still
// gives about 32K waves (half of them fall beyond the triangle's diagonal;
// level 11 on 8 triangles: 16 rows, 152 GDoF/s FP64 against 127 with 64 rows).
// OP 0: scaled rows; OP 1: nodal rows (the six incident elements from the
// same seven values, element matrices of the triangle in Aall).
template <typename T, int OP>
__global__ __launch_bounds__(B2) void k2d_march(int n, int64_t Spad, int n_seg, int jc, const T *__restrict__ w,
                                                const double *__restrict__ Aall, const T *__restrict__ k,
                                                const T *__restrict__ u, T *__restrict__ y)
{
    const int wv = blockIdx.x * (B2 / 64) + (threadIdx.x >> 6);
    const int chunks = (n - 2 + jc - 1) / jc;
    if (wv >= n_seg * chunks) return;
    const int seg = wv % n_seg, ch = wv / n_seg;
    const int lane = threadIdx.x & 63;
    const int j0 = 1 + ch * jc, j1 = min(n - 2, j0 + jc - 1);
    const int i0 = 1 + 62 * seg;
    if (i0 > n - 1 - j0) return;  // the whole wave lies beyond the rows' ends (uniform per wave)
    const int col = i0 - 1 + lane;
    const int tri = blockIdx.y;
    const T *ub = u + (int64_t)tri * Spad, *kb = k + (int64_t)tri * Spad;
    T *yb = y + (int64_t)tri * Spad;
    const T w0 = w[tri * 3], w1 = w[tri * 3 + 1], w2 = w[tri * 3 + 2];
    // value of row r at this lane's column (0 outside the lattice)
    auto rs = [&](int r) { return (int64_t)r * (n + 1) - (int64_t)r * (r - 1) / 2; };
    auto ld = [&](const T *a, int r) { return (r >= 0 && r <= n && col <= n - r) ? a[rs(r) + col] : T(0); };
    T um = ld(ub, j0 - 1), uc = ld(ub, j0), up = ld(ub, j0 + 1);
    T km = ld(kb, j0 - 1), kc = ld(kb, j0), kp = ld(kb, j0 + 1);
    for (int j = j0; j <= j1; ++j) {
        // prefetch row j+2 before the shuffles of row j
        const T un = ld(ub, j + 2), kn = ld(kb, j + 2);
        const T ue = __shfl_down(uc, 1, 64), uw = __shfl_up(uc, 1, 64);
        const T ke = __shfl_down(kc, 1, 64), kw = __shfl_up(kc, 1, 64);
        const T unw = __shfl_up(up, 1, 64), knw = __shfl_up(kp, 1, 64);   // (i-1, j+1)
        const T use = __shfl_down(um, 1, 64), kse = __shfl_down(km, 1, 64);  // (i+1, j-1)
        if (lane >= 1 && lane <= 62 && col >= 1 && col <= n - 1 - j) {
            if (OP == 0) {
                const T a0 = (kc + ke) * (ue - uc) + (kc + kw) * (uw - uc);
                const T a1 = (kc + kp) * (up - uc) + (kc + km) * (um - uc);
                const T a2 = (kc + knw) * (unw - uc) + (kc + kse) * (use - uc);
                yb[rs(j) + col] = w0 * a0 + w1 * a1 + w2 * a2;
            } else {
                // neighbours in D2 order, centre last
                const T uu[7] = {ue, up, unw, uw, um, use, uc};
                const T kk[7] = {ke, kp, knw, kw, km, kse, kc};
                const double *A = Aall + tri * 9;
                T acc = T(0);
#pragma unroll
                for (int e = 0; e < 6; ++e) {
                    int idx[3];
#pragma unroll
                    for (int v = 0; v < 3; ++v) {
                        const int di = AROUND[e].off[v][0], dj = AROUND[e].off[v][1];
                        idx[v] = (di == 0 && dj == 0) ? 6 : dir_of(di, dj);
                    }
                    const int me = AROUND[e].me;
                    const T kbar = (kk[idx[0]] + kk[idx[1]] + kk[idx[2]]) / T(3);
                    T r = T(0);
#pragma unroll
                    for (int v = 0; v < 3; ++v)
                        if (v != me) r += (T)A[me * 3 + v] * (uu[idx[v]] - uc);
                    acc += kbar * r;
                }
                yb[rs(j) + col] = acc;
            }
        }
        um = uc; uc = up; up = un;
        km = kc; kc = kp; kp = kn;
    }
}

// after the interior kernel, one launch for the rest of the rows (disjoint
// slot sets): threads [0, n_sh) shared rows from merged coefficients, written
// to every copy; [n_sh, n_sh + n_corr) the MA2 corrections of interior rows;
// then the Dirichlet slots (set to 0)
template <typename T>
__global__ __launch_bounds__(B2) void k2d_tail(int n_sh, const int32_t *__restrict__ eoff,
                                               const int64_t *__restrict__ nbs, const T *__restrict__ coef,
                                               const int64_t *__restrict__ self, const int32_t *__restrict__ coff,
                                               const int64_t *__restrict__ cslot, int64_t n_corr,
                                               const int64_t *__restrict__ crow, const int64_t *__restrict__ cnb,
                                               const T *__restrict__ cdl, int64_t n_dir,
                                               const int64_t *__restrict__ dslots, const T *__restrict__ u,
                                               T *__restrict__ y)
{
    int64_t q = (int64_t)blockIdx.x * B2 + threadIdx.x;
    if (q < n_sh) {
        const T u0 = u[self[q]];
        T acc = T(0);
        for (int e = eoff[q]; e < eoff[q + 1]; ++e) acc += coef[e] * (u[nbs[e]] - u0);
        for (int c = coff[q]; c < coff[q + 1]; ++c) y[cslot[c]] = acc;
        return;
    }
    q -= n_sh;
    if (q < n_corr) {
        const int64_t a = crow[q];
        const T u0 = u[a];
        y[a] += cdl[2 * q] * (u[cnb[2 * q]] - u0) + cdl[2 * q + 1] * (u[cnb[2 * q + 1]] - u0);
        return;
    }
    q -= n_corr;
    if (q < n_dir) y[dslots[q]] = T(0);
}

template <typename T>
__global__ void k2d_from_canon(int64_t n_slots, const int64_t *__restrict__ s2c, const T *__restrict__ vc,
                               T *__restrict__ vs)
{
    const int64_t q = (int64_t)blockIdx.x * B2 + threadIdx.x;
    if (q >= n_slots) return;
    const int64_t c = s2c[q];
    vs[q] = c >= 0 ? vc[c] : T(0);
}
template <typename T>
__global__ void k2d_to_canon(int64_t n_nodes, const int64_t *__restrict__ c2s, const T *__restrict__ vs,
                             T *__restrict__ vc)
{
    const int64_t q = (int64_t)blockIdx.x * B2 + threadIdx.x;
    if (q < n_nodes) vc[q] = vs[c2s[q]];
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + B2 - 1) / B2); }

template <typename T>
struct Dev2 {
    const T *w, *k, *cs, *cn, *dl;
};

template <typename T>
hhg_status apply_t(hhg2d_ctx c, int op, const T *u, T *y, hipStream_t st, const Dev2<T> &D)
{
    const int n = c->n;
    if (n >= 3) {
        const int n_seg = (n - 1 + 61) / 62;
        int jc = 64;
        while (jc > 8 && (int64_t)n_seg * ((n - 2 + jc - 1) / jc) * c->nt < 32768) jc /= 2;
        const int chunks = (n - 2 + jc - 1) / jc;
        const dim3 g((unsigned)((n_seg * chunks + B2 / 64 - 1) / (B2 / 64)), (unsigned)c->nt);
        if (op == 0) k2d_march<T, 0><<<g, B2, 0, st>>>(n, c->Spad, n_seg, jc, D.w, c->d_A, D.k, u, y);
        else k2d_march<T, 1><<<g, B2, 0, st>>>(n, c->Spad, n_seg, jc, D.w, c->d_A, D.k, u, y);
    }
    const int64_t n_corr = op == 0 ? c->n_corr : 0, n_dir = (int64_t)c->dir_slots.size();
    const int64_t n_tail = c->n_sh + n_corr + n_dir;
    if (n_tail)
        k2d_tail<T><<<nblk(n_tail), B2, 0, st>>>(c->n_sh, c->d_sh_eoff, c->d_sh_nb, op == 0 ? D.cs : D.cn,
                                                 c->d_sh_self, c->d_sh_off, c->d_sh_cslot, n_corr, c->d_c_row,
                                                 c->d_c_nb, D.dl, n_dir, c->d_dir, u, y);
    HIP2(c, hipGetLastError());
    return HHG_OK;
}

// node key: sorted (macro vertex, weight) pairs with non-zero weight
struct Key2 {
    int v[3], w[3];
    bool operator<(const Key2 &o) const
    {
        for (int a = 0; a < 3; ++a) {
            if (v[a] != o.v[a]) return v[a] < o.v[a];
            if (w[a] != o.w[a]) return w[a] < o.w[a];
        }
        return false;
    }
};
Key2 key_of(const hhg2d_ctx c, int t, int i, int j)
{
    const int n = c->n, w[3] = {n - i - j, i, j};
    std::pair<int, int> p[3];
    int m = 0;
    for (int a = 0; a < 3; ++a)
        if (w[a] > 0) p[m++] = {c->T[3 * t + a], w[a]};
    std::sort(p, p + m);
    Key2 K;
    for (int a = 0; a < 3; ++a) {
        K.v[a] = a < m ? p[a].first : -1;
        K.w[a] = a < m ? p[a].second : 0;
    }
    return K;
}

hhg_status build2d(hhg2d_ctx c)
{
    const int n = c->n, nt = c->nt;
    c->S = (int64_t)(n + 1) * (n + 2) / 2;
    c->Spad = (c->S + 63) / 64 * 64;
    c->n_slots = (int64_t)nt * c->Spad;
    // macro element matrices, weights, lambda_min
    c->A.assign((size_t)nt * 9, 0.0);
    c->lam.assign(nt, 0.0);
    std::vector<double> w((size_t)nt * 3);
    for (int t = 0; t < nt; ++t) {
        double P[3][2], A[3][3];
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 2; ++d) P[a][d] = c->X[2 * c->T[3 * t + a] + d];
        if (!element_matrix(P, A)) return fail2(c, HHG_EMESH, "triangle %d is degenerate", t);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) c->A[(size_t)t * 9 + a * 3 + b] = A[a][b];
        for (int d = 0; d < 3; ++d) w[(size_t)t * 3 + d] = A[PAIR[d][0]][PAIR[d][1]];
        c->lam[t] = lambda_min_T(A);
    }
    // macro boundary edges (one triangle)
    std::map<std::pair<int, int>, int> ecount;
    for (int t = 0; t < nt; ++t)
        for (int a = 0; a < 3; ++a) {
            int p = c->T[3 * t + a], q = c->T[3 * t + (a + 1) % 3];
            ecount[{std::min(p, q), std::max(p, q)}]++;
        }
    auto bnd_edge = [&](int p, int q) { auto it = ecount.find({std::min(p, q), std::max(p, q)}); return it != ecount.end() && it->second == 1; };
    // nodes: a triangle's interior positions have one copy and get their id
    // directly; positions on its edges are identified across triangles by key
    std::map<Key2, int64_t> ids;
    std::map<int64_t, std::vector<std::pair<int, int>>> multi;  // copies of edge / vertex nodes
    c->slot2canon.assign((size_t)c->n_slots, -1);
    int64_t next = 0;
    auto add_node = [&](int t, int i, int j, bool dir) {
        const double w0 = (double)(n - i - j) / n, w1 = (double)i / n, w2 = (double)j / n;
        for (int d = 0; d < 2; ++d)
            c->node_xy.push_back(w0 * c->X[2 * c->T[3 * t] + d] + w1 * c->X[2 * c->T[3 * t + 1] + d] +
                                 w2 * c->X[2 * c->T[3 * t + 2] + d]);
        c->dir_node.push_back(dir ? 1 : 0);
        c->canon2slot.push_back((int64_t)t * c->Spad + slot_of(n, i, j));
        return next++;
    };
    for (int t = 0; t < nt; ++t)
        for (int j = 0; j <= n; ++j)
            for (int i = 0; i + j <= n; ++i) {
                const int64_t gs = (int64_t)t * c->Spad + slot_of(n, i, j);
                if (i > 0 && j > 0 && i + j < n) {
                    c->slot2canon[gs] = add_node(t, i, j, false);
                    continue;
                }
                const Key2 K = key_of(c, t, i, j);
                auto it = ids.find(K);
                int64_t id;
                if (it == ids.end()) {
                    int m = 0;
                    while (m < 3 && K.v[m] >= 0) ++m;
                    bool dir = false;
                    if (m == 1) {
                        for (auto &e : ecount)
                            if (e.second == 1 && (e.first.first == K.v[0] || e.first.second == K.v[0])) dir = true;
                    } else {
                        dir = bnd_edge(K.v[0], K.v[1]);
                    }
                    id = add_node(t, i, j, dir);
                    ids.emplace(K, id);
                } else {
                    id = it->second;
                }
                multi[id].push_back({t, (int)slot_of(n, i, j)});
                c->slot2canon[gs] = id;
            }
    c->n_nodes = next;
    c->n_unknowns = 0;
    for (int64_t q = 0; q < c->n_nodes; ++q)
        if (!c->dir_node[q]) ++c->n_unknowns;
    // Dirichlet copies, and shared rows: the non-Dirichlet nodes of interior
    // macro edges and vertices (several copies; an edge / vertex node with one
    // copy lies on the boundary and is Dirichlet)
    c->sh.off.assign(1, 0);
    for (auto &kv : multi) {
        const int64_t q = kv.first;
        if (c->dir_node[q]) {
            for (auto &cp : kv.second) c->dir_slots.push_back((int64_t)cp.first * c->Spad + cp.second);
            continue;
        }
        if (kv.second.size() < 2) return fail2(c, HHG_EMESH, "a boundary node is not on a boundary edge");
        c->sh.self.push_back(c->canon2slot[q]);
        c->sh.copy.push_back(kv.second);
        for (auto &cp : kv.second) c->sh.cslot.push_back((int64_t)cp.first * c->Spad + cp.second);
        c->sh.off.push_back((int32_t)c->sh.cslot.size());
    }
    c->n_sh = (int)c->sh.self.size();
    // device arrays of the layout
    std::vector<float> w32(w.begin(), w.end());
    TRY2(upload2(c, &c->w64, w));
    TRY2(upload2(c, &c->w32, w32));
    TRY2(upload2(c, &c->d_A, c->A));
    TRY2(upload2(c, &c->d_s2c, c->slot2canon));
    TRY2(upload2(c, &c->d_c2s, c->canon2slot));
    TRY2(upload2(c, &c->d_dir, c->dir_slots));
    TRY2(upload2(c, &c->d_sh_self, c->sh.self));
    TRY2(upload2(c, &c->d_sh_off, c->sh.off));
    TRY2(upload2(c, &c->d_sh_cslot, c->sh.cslot));
    TRY2(dalloc2(c, &c->k64, c->n_slots));
    TRY2(dalloc2(c, &c->k32, c->n_slots));
    return HHG_OK;
}

// position (i, j) of a slot
inline void pos_of(int n, int s, int &i, int &j)
{
    // slot(0, j) = j (2n + 3 - j) / 2: the root of the quadratic, then exact
    const double b = 2.0 * n + 3.0;
    j = (int)((b - std::sqrt(std::max(0.0, b * b - 8.0 * s))) / 2.0);
    j = std::max(0, std::min(j, n));
    while (j > 0 && slot_of(n, 0, j) > s) --j;
    while (j < n && slot_of(n, 0, j + 1) <= s) ++j;
    i = s - (int)slot_of(n, 0, j);
}

// the scaled factor of lattice edge (a, b) inside macro triangle t: (k_a +
// k_b)/2, or k_mod where MA2 (Sec. 4.1) triggers for a gray edge
double edge_factor(const hhg2d_ctx c, int t, int ai, int aj, int bi, int bj, bool modify)
{
    const int n = c->n;
    const double *kb = c->k_slot.data() + (size_t)t * c->Spad;
    auto kat = [&](int i, int j) { return kb[slot_of(n, i, j)]; };
    const double ke = 0.5 * (kat(ai, aj) + kat(bi, bj));
    if (!modify) return ke;
    const int d = dir_of(bi - ai, bj - aj);
    const double a12 = c->A[(size_t)t * 9 + PAIR[d][0] * 3 + PAIR[d][1]];
    if (!(a12 > 0)) return ke;
    // the elements of t holding the edge; k_{e;min} over their edges
    double kmin = INFINITY;
    int nel = 0;
    for (int e = 0; e < 6; ++e) {
        int vi[3], vj[3];
        bool ok = true, has_b = false;
        for (int v = 0; v < 3; ++v) {
            vi[v] = ai + AROUND[e].off[v][0];
            vj[v] = aj + AROUND[e].off[v][1];
            ok = ok && in_tri(n, vi[v], vj[v]);
            has_b = has_b || (vi[v] == bi && vj[v] == bj);
        }
        if (!ok || !has_b) continue;
        ++nel;
        for (int p = 0; p < 3; ++p)
            for (int q = p + 1; q < 3; ++q) kmin = std::min(kmin, 0.5 * (kat(vi[p], vj[p]) + kat(vi[q], vj[q])));
    }
    if (!nel) return ke;
    if ((ke - kmin) * a12 > kmin * c->lam[t]) return kmin * (1.0 + c->lam[t] / a12);
    return ke;
}

hhg_status set_coef2d(hhg2d_ctx c, const double *k)
{
    const int n = c->n, nt = c->nt;
    for (int64_t q = 0; q < c->n_nodes; ++q)
        if (!(k[q] > 0) || !std::isfinite(k[q]))
            return fail2(c, HHG_ECOEF, "coefficient must be positive and finite (node %lld)", (long long)q);
    c->k_slot.assign((size_t)c->n_slots, 1.0);
    for (int64_t s = 0; s < c->n_slots; ++s)
        if (c->slot2canon[s] >= 0) c->k_slot[s] = k[c->slot2canon[s]];
    const bool modify = !(c->flags & HHG2D_FLAG_NO_MODIFICATION);
    c->n_mod = 0;
    // shared rows: merged entries over the elements of every copy
    std::vector<int32_t> eoff(1, 0);
    std::vector<int64_t> nbs;
    std::vector<double> cs, cn;
    for (int q = 0; q < c->n_sh; ++q) {
        std::map<int64_t, int> ent;  // neighbour canonical id -> entry
        const size_t e0 = nbs.size();
        for (auto &cp : c->sh.copy[q]) {
            const int t = cp.first;
            int ai, aj;
            pos_of(n, cp.second, ai, aj);
            const double *A = c->A.data() + (size_t)t * 9;
            const double *kb = c->k_slot.data() + (size_t)t * c->Spad;
            for (int e = 0; e < 6; ++e) {
                int vi[3], vj[3];
                bool ok = true;
                for (int v = 0; v < 3; ++v) {
                    vi[v] = ai + AROUND[e].off[v][0];
                    vj[v] = aj + AROUND[e].off[v][1];
                    ok = ok && in_tri(n, vi[v], vj[v]);
                }
                if (!ok) continue;
                const int me = AROUND[e].me;
                double kbar = 0;
                for (int v = 0; v < 3; ++v) kbar += kb[slot_of(n, vi[v], vj[v])];
                kbar /= 3.0;
                for (int v = 0; v < 3; ++v) {
                    if (v == me) continue;
                    const int64_t gs = (int64_t)t * c->Spad + slot_of(n, vi[v], vj[v]);
                    const int64_t id = c->slot2canon[gs];
                    auto it = ent.find(id);
                    int m;
                    if (it == ent.end()) {
                        m = (int)(nbs.size() - e0);
                        ent.emplace(id, m);
                        nbs.push_back(gs);
                        cs.push_back(0.0);
                        cn.push_back(0.0);
                    } else {
                        m = it->second;
                    }
                    const double f = edge_factor(c, t, ai, aj, vi[v], vj[v], modify);
                    cs[e0 + m] += A[me * 3 + v] * f;
                    cn[e0 + m] += A[me * 3 + v] * kbar;
                }
            }
        }
        eoff.push_back((int32_t)nbs.size());
    }
    // MA2 corrections of interior rows: gray directions of each triangle
    std::vector<int64_t> crow, cnb;
    std::vector<double> cdl;
    if (modify)
        for (int t = 0; t < nt; ++t) {
            int gd = -1;
            for (int d = 0; d < 3; ++d)
                if (c->A[(size_t)t * 9 + PAIR[d][0] * 3 + PAIR[d][1]] > 0) gd = d;
            if (gd < 0) continue;
            const double a12 = c->A[(size_t)t * 9 + PAIR[gd][0] * 3 + PAIR[gd][1]];
            const double *kb = c->k_slot.data() + (size_t)t * c->Spad;
            for (int j = 1; j <= n - 2; ++j)
                for (int i = 1; i + j <= n - 1; ++i) {
                    int64_t nb2[2] = {0, 0};
                    double dl[2] = {0, 0};
                    bool any = false;
                    for (int h = 0; h < 2; ++h) {
                        const int d = gd + 3 * h;
                        const int bi = i + D2[d][0], bj = j + D2[d][1];
                        nb2[h] = (int64_t)t * c->Spad + slot_of(n, bi, bj);
                        const double ke = 0.5 * (kb[slot_of(n, i, j)] + kb[slot_of(n, bi, bj)]);
                        const double f = edge_factor(c, t, i, j, bi, bj, true);
                        if (f != ke) {
                            // both elements of t holding an edge from an interior node
                            dl[h] = 2.0 * a12 * (f - ke);
                            any = true;
                        }
                    }
                    if (any) {
                        crow.push_back((int64_t)t * c->Spad + slot_of(n, i, j));
                        cnb.push_back(nb2[0]);
                        cnb.push_back(nb2[1]);
                        cdl.push_back(dl[0]);
                        cdl.push_back(dl[1]);
                    }
                }
        }
    c->n_corr = (int64_t)crow.size();
    // triggered gray edges, each once
    if (modify)
        for (int t = 0; t < nt; ++t) {
            int gd = -1;
            for (int d = 0; d < 3; ++d)
                if (c->A[(size_t)t * 9 + PAIR[d][0] * 3 + PAIR[d][1]] > 0) gd = d;
            if (gd < 0) continue;
            const double *kb = c->k_slot.data() + (size_t)t * c->Spad;
            for (int j = 0; j <= n; ++j)
                for (int i = 0; i + j <= n; ++i) {
                    const int bi = i + D2[gd][0], bj = j + D2[gd][1];
                    if (!in_tri(n, bi, bj)) continue;
                    const double ke = 0.5 * (kb[slot_of(n, i, j)] + kb[slot_of(n, bi, bj)]);
                    if (edge_factor(c, t, i, j, bi, bj, true) != ke) ++c->n_mod;
                }
        }
    // upload (shared entries and corrections are rebuilt per coefficient)
    for (void *p : {(void *)c->d_sh_eoff, (void *)c->d_sh_nb, (void *)c->d_sh_cs64, (void *)c->d_sh_cn64,
                    (void *)c->d_sh_cs32, (void *)c->d_sh_cn32, (void *)c->d_c_row, (void *)c->d_c_nb,
                    (void *)c->d_c_dl64, (void *)c->d_c_dl32}) {
        if (!p) continue;
        auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
        if (it != c->allocs.end()) c->allocs.erase(it);
        (void)hipFree(p);
    }
    c->d_sh_eoff = nullptr; c->d_sh_nb = nullptr; c->d_sh_cs64 = nullptr; c->d_sh_cn64 = nullptr;
    c->d_sh_cs32 = nullptr; c->d_sh_cn32 = nullptr; c->d_c_row = nullptr; c->d_c_nb = nullptr;
    c->d_c_dl64 = nullptr; c->d_c_dl32 = nullptr;
    std::vector<float> cs32(cs.begin(), cs.end()), cn32(cn.begin(), cn.end()), cdl32(cdl.begin(), cdl.end());
    TRY2(upload2(c, &c->d_sh_eoff, eoff));
    TRY2(upload2(c, &c->d_sh_nb, nbs));
    TRY2(upload2(c, &c->d_sh_cs64, cs));
    TRY2(upload2(c, &c->d_sh_cn64, cn));
    TRY2(upload2(c, &c->d_sh_cs32, cs32));
    TRY2(upload2(c, &c->d_sh_cn32, cn32));
    TRY2(upload2(c, &c->d_c_row, crow));
    TRY2(upload2(c, &c->d_c_nb, cnb));
    TRY2(upload2(c, &c->d_c_dl64, cdl));
    TRY2(upload2(c, &c->d_c_dl32, cdl32));
    std::vector<float> k32(c->k_slot.begin(), c->k_slot.end());
    HIP2(c, hipMemcpy(c->k64, c->k_slot.data(), c->n_slots * 8, hipMemcpyHostToDevice));
    HIP2(c, hipMemcpy(c->k32, k32.data(), c->n_slots * 4, hipMemcpyHostToDevice));
    c->have_k = true;
    return HHG_OK;
}

}  // namespace

extern "C" {

hhg_status hhg2d_create(const double *xy, int32_t n_vert, const int32_t *tri, int32_t n_tri, int32_t level,
                        uint32_t flags, hhg2d_ctx *out)
{
    if (!out) return HHG_EINVAL;
    *out = nullptr;
    // one grid row of blocks per triangle: at most 65535 triangles
    if (!xy || !tri || n_vert < 3 || n_tri < 1 || n_tri > 65535 || level < 0 || level > 13) return HHG_EINVAL;
    for (int64_t q = 0; q < 3 * (int64_t)n_tri; ++q)
        if (tri[q] < 0 || tri[q] >= n_vert) return HHG_EMESH;
    hhg2d_ctx c = new hhg2d_ctx_s;
    c->level = level;
    c->n = 1 << level;
    c->nt = n_tri;
    c->flags = flags;
    c->X.assign(xy, xy + 2 * (size_t)n_vert);
    c->T.assign(tri, tri + 3 * (size_t)n_tri);
    const hhg_status s = build2d(c);
    if (s != HHG_OK) {
        hhg2d_destroy(c);
        return s;
    }
    *out = c;
    return HHG_OK;
}

hhg_status hhg2d_destroy(hhg2d_ctx c)
{
    if (!c) return HHG_OK;
    (void)hipDeviceSynchronize();
    for (void *p : c->allocs) (void)hipFree(p);
    delete c;
    return HHG_OK;
}

const char *hhg2d_last_error(hhg2d_ctx c) { return c ? c->err.c_str() : ""; }

hhg_status hhg2d_sizes(hhg2d_ctx c, int64_t *n_slots, int64_t *n_nodes, int64_t *n_unknowns, int64_t *n_modified)
{
    if (!c) return HHG_EINVAL;
    if (n_slots) *n_slots = c->n_slots;
    if (n_nodes) *n_nodes = c->n_nodes;
    if (n_unknowns) *n_unknowns = c->n_unknowns;
    if (n_modified) *n_modified = c->n_mod;
    return HHG_OK;
}

hhg_status hhg2d_node_coords(hhg2d_ctx c, double *xy, uint8_t *dirichlet)
{
    if (!c) return HHG_EINVAL;
    if (xy) std::memcpy(xy, c->node_xy.data(), c->node_xy.size() * sizeof(double));
    if (dirichlet) std::memcpy(dirichlet, c->dir_node.data(), c->dir_node.size());
    return HHG_OK;
}

hhg_status hhg2d_set_coefficient(hhg2d_ctx c, const double *k)
{
    if (!c || !k) return fail2(c, HHG_EINVAL, "NULL argument");
    return set_coef2d(c, k);
}

hhg_status hhg2d_from_canonical(hhg2d_ctx c, hhg_dtype dt, const void *v_canon, void *v_slots, void *stream)
{
    if (!c || !v_canon || !v_slots) return fail2(c, HHG_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    if (dt == HHG_F64)
        k2d_from_canon<double><<<nblk(c->n_slots), B2, 0, st>>>(c->n_slots, c->d_s2c, (const double *)v_canon,
                                                                (double *)v_slots);
    else if (dt == HHG_F32)
        k2d_from_canon<float><<<nblk(c->n_slots), B2, 0, st>>>(c->n_slots, c->d_s2c, (const float *)v_canon,
                                                               (float *)v_slots);
    else return fail2(c, HHG_EINVAL, "bad dtype");
    HIP2(c, hipGetLastError());
    return HHG_OK;
}

hhg_status hhg2d_to_canonical(hhg2d_ctx c, hhg_dtype dt, const void *v_slots, void *v_canon, void *stream)
{
    if (!c || !v_canon || !v_slots) return fail2(c, HHG_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    if (dt == HHG_F64)
        k2d_to_canon<double><<<nblk(c->n_nodes), B2, 0, st>>>(c->n_nodes, c->d_c2s, (const double *)v_slots,
                                                              (double *)v_canon);
    else if (dt == HHG_F32)
        k2d_to_canon<float><<<nblk(c->n_nodes), B2, 0, st>>>(c->n_nodes, c->d_c2s, (const float *)v_slots,
                                                             (float *)v_canon);
    else return fail2(c, HHG_EINVAL, "bad dtype");
    HIP2(c, hipGetLastError());
    return HHG_OK;
}

static hhg_status apply2d(hhg2d_ctx c, int op, hhg_dtype dt, const void *u, void *y, void *stream)
{
    if (!c) return HHG_EINVAL;
    if (!c->have_k) return fail2(c, HHG_ESTATE, "no coefficient set");
    if (!u || !y || u == y) return fail2(c, HHG_EINVAL, "u and y must be distinct non-NULL vectors");
    hipStream_t st = (hipStream_t)stream;
    if (dt == HHG_F64)
        return apply_t<double>(c, op, (const double *)u, (double *)y, st,
                               Dev2<double>{c->w64, c->k64, c->d_sh_cs64, c->d_sh_cn64, c->d_c_dl64});
    if (dt == HHG_F32)
        return apply_t<float>(c, op, (const float *)u, (float *)y, st,
                              Dev2<float>{c->w32, c->k32, c->d_sh_cs32, c->d_sh_cn32, c->d_c_dl32});
    return fail2(c, HHG_EINVAL, "bad dtype");
}

hhg_status hhg2d_apply_scaled(hhg2d_ctx c, hhg_dtype dt, const void *u, void *y, void *stream)
{
    return apply2d(c, 0, dt, u, y, stream);
}

hhg_status hhg2d_apply_nodal(hhg2d_ctx c, hhg_dtype dt, const void *u, void *y, void *stream)
{
    return apply2d(c, 1, dt, u, y, stream);
}

}  // extern "C"
