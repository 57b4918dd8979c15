// hhg_kernels.hip -- HIP kernels for gfx950 (MI355X): scaled-stencil and
// nodal-integration operator application on tetrahedral-index lattices,
// residual norms, smoother updates, grid transfer and the coarse solve.
//
// Work decomposition.  Slot vectors hold one closed tet lattice per macro tet
// (planes k in turn, inside a plane the anti-diagonals i + j in turn).
// Interior rows are computed by column marching (k_march2 for the scaled
// operator, two rows per lane; k_march for the nodal one): a wave owns a run
// of consecutive in-plane offsets, walks a chunk of planes with three planes
// held in registers, and takes the i +- 1 neighbours from the adjacent lanes.
// Rows of nodes on primitives shared by several tets (macro faces, edges,
// vertices) come from merged neighbour lists built once per coefficient
// field (k_shared_rows) and are written to every copy, so every slot vector
// stays consistent.  Extra blocks of the marching launches write 0 to the
// Dirichlet slots.  Marching grids are remapped so that each of the 8 XCDs
// walks one contiguous eighth of the work items (neighbouring diagonals of
// the same planes then meet in that XCD's L2).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "hhg_internal.h"
#include "hhg_lattice.h"
#include "hhg_march.h"

namespace hhg {

// ---------------------------------------------------------------- helpers
// (i,j,k) of slot s of a tet lattice with n intervals (n <= 1024)
__device__ __forceinline__ void decode_slot(int n, int s, int &i, int &j, int &k)
{
    const int q = tc32(n) - s;  // slots in planes >= k, counted from the top
    int m = (int)(cbrtf(6.0f * (float)q)) - 2;
    m = m < 0 ? 0 : m;
    while (tc32(m) < q) ++m;
    while (m > 0 && tc32(m - 1) >= q) --m;
    k = n - m;
    const int t = s - (tc32(n) - tc32(m));  // offset inside the plane
    int d = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((d + 1) * (d + 2) / 2 <= t) ++d;
    while (d > 0 && d * (d + 1) / 2 > t) --d;
    i = t - d * (d + 1) / 2;
    j = d - i;
}

// slots of the 14 neighbours of slot s = (i,j,k) in DIR order; sd = i + j,
// m = n - k.  Plane k holds tr32(m) slots, plane k-1 tr32(m+1); the
// anti-diagonal s+1 starts s+1 slots after the start of diagonal s.
__device__ __forceinline__ void neighbour_slots(int s, int sd, int m, int nb[NDIR])
{
    const int up = s + tr32(m);        // (i, j, k+1)
    const int dn = s - tr32(m + 1);    // (i, j, k-1)
    nb[0] = s + sd + 2;                // ( 1, 0, 0)
    nb[1] = s + sd + 1;                // ( 0, 1, 0)
    nb[2] = up;                        // ( 0, 0, 1)
    nb[3] = s + 1;                     // ( 1,-1, 0)
    nb[4] = dn + sd + 2;               // ( 1, 0,-1)
    nb[5] = dn + sd + 1;               // ( 0, 1,-1)
    nb[6] = up + 1;                    // ( 1,-1, 1)
    nb[7] = s - sd - 1;                // (-1, 0, 0)
    nb[8] = s - sd;                    // ( 0,-1, 0)
    nb[9] = dn;                        // ( 0, 0,-1)
    nb[10] = s - 1;                    // (-1, 1, 0)
    nb[11] = up - sd - 1;              // (-1, 0, 1)
    nb[12] = up - sd;                  // ( 0,-1, 1)
    nb[13] = dn - 1;                   // (-1, 1,-1)
}

__device__ __forceinline__ double warp_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ double warp_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}
// block-wide sum (op_max = 0) or max (op_max = 1); result valid in thread 0
__device__ __forceinline__ double block_reduce(double v, int op_max)
{
    __shared__ double red[BLOCK / 64];
    v = op_max ? warp_max(v) : warp_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < BLOCK / 64; ++q) v = op_max ? fmax(v, red[q]) : v + red[q];
    }
    return v;
}

static inline int volume_grid(int n_tet, int bpt)
{
    const int nb = n_tet * bpt;
    return ((nb + 7) / 8) * 8;
}

static inline int blocks_for(int64_t n) { return (int)((n + BLOCK - 1) / BLOCK); }

// element vertex directions: ELEM_DIR[t][a][b] = direction index of vertex b
// of element shape t seen from its vertex a (14 when a == b)
struct ElemDirTable {
    int v[NTYPE][4][4];
    constexpr ElemDirTable() : v()
    {
        for (int t = 0; t < NTYPE; ++t)
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b)
                    v[t][a][b] = dir_index(TYPE_OFF[t][b][0] - TYPE_OFF[t][a][0],
                                           TYPE_OFF[t][b][1] - TYPE_OFF[t][a][1],
                                           TYPE_OFF[t][b][2] - TYPE_OFF[t][a][2]);
    }
};
constexpr ElemDirTable ELEM_DIR{};

// ---------------------------------------------------------------- interior rows
// Interior rows by column marching.  One wave takes 64 consecutive in-plane
// offsets t (the same (i,j) columns in every plane; lanes 1..62 produce rows,
// lanes 0 and 63 only feed their neighbours) and walks the planes k0..k1.  At
// plane k a row needs, per array, the anti-diagonals s-1, s, s+1 of planes
// k-1, k, k+1 at positions i-1..i+1.  Positions i+-1 come from the adjacent
// lanes (interior nodes never sit at a diagonal's end), and the planes roll
// through registers, so each step loads three coalesced values per array:
// diagonals s-1, s, s+1 of plane k+1 at position i.
//
// OP 0: scaled stencil  y_i = sum_d w_d (k_i + k_{i+d}) (u_{i+d} - u_i)
//       (Sec. 6.1 with the difference form of Sec. 6.3; w_d = shat_d / 2);
// OP 1: nodal integration y_i = sum_{t contains i} kbar_t sum_b A_t[i,b](u_b - u_i)
//       (eq. (standardfe): 24 elements, kbar_t the mean vertex value of k).
// Extra blocks after the interior ones write 0 to Dirichlet boundary slots.

template <typename T, int OP>
__device__ __forceinline__ T row_value(const T uu[NDIR + 1], const T kk[NDIR + 1], const T *__restrict__ w)
{
    const T u0 = uu[NDIR], k0 = kk[NDIR];
    T acc = T(0);
    if (OP == 0) {
#pragma unroll
        for (int d = 0; d < NDIR; ++d) acc += w[d] * (k0 + kk[d]) * (uu[d] - u0);
    } else {
        // per direction d: C_d = sum over the incident elements t holding the
        // edge (node, node + d) of (sum of k at t's vertices) (A_t / 4)[a, b];
        // then y = sum_d C_d (u_d - u_0)
        T cd[NDIR];
#pragma unroll
        for (int d = 0; d < NDIR; ++d) cd[d] = T(0);
#pragma unroll
        for (int t = 0; t < NTYPE; ++t)
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int d0 = ELEM_DIR.v[t][a][0], d1 = ELEM_DIR.v[t][a][1];
                const int d2 = ELEM_DIR.v[t][a][2], d3 = ELEM_DIR.v[t][a][3];
                const T ks = (kk[d0] + kk[d1]) + (kk[d2] + kk[d3]);
                const T *e = w + t * 16 + a * 4;
                if (d0 != NDIR) cd[d0 < NDIR ? d0 : 0] += ks * e[0];
                if (d1 != NDIR) cd[d1 < NDIR ? d1 : 0] += ks * e[1];
                if (d2 != NDIR) cd[d2 < NDIR ? d2 : 0] += ks * e[2];
                if (d3 != NDIR) cd[d3 < NDIR ? d3 : 0] += ks * e[3];
            }
#pragma unroll
        for (int d = 0; d < NDIR; ++d) acc += cd[d] * (uu[d] - u0);
    }
    return acc;
}

// scaled row with the weights of opposite directions paired (interior
// stencils have w_d = w_{d+7}):
//   y = sum_{d<7} w_d [(k0 + k_d)(u_d - u0) + (k0 + k_{d+7})(u_{d+7} - u0)]
template <typename T>
__device__ __forceinline__ T scaled_row_paired(const T uu[NDIR + 1], const T kk[NDIR + 1], const T wr[NDIR / 2])
{
    const T u0 = uu[NDIR], k0 = kk[NDIR];
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < NDIR / 2; ++d) {
        const T a = (k0 + kk[d + NDIR / 2]) * (uu[d + NDIR / 2] - u0);
        acc += wr[d] * ((k0 + kk[d]) * (uu[d] - u0) + a);
    }
    return acc;
}

// an empty register-to-register asm: the value passes unchanged, but the
// compiler can no longer prove it equal to its earlier self, so lane shifts
// of it are recomputed where used instead of being held in registers
template <typename T>
__device__ __forceinline__ void renew(T &v)
{
    asm("" : "+v"(v));
}
template <typename T>
__device__ __forceinline__ void mplane_renew(MPlane<T> &p)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        renew(p.u[c]);
        renew(p.k[c]);
    }
}

// PF: planes in flight ahead of the ones in use; WPE: waves per SIMD the
// register budget must allow; SH 0 holds a plane's lane-shifted copies for
// the two steps that use them, SH 1 recomputes them at each use (fewer
// registers, more lane moves).  NS = PF + 3 register sets rotate through the
// roles plane k-1, k, k+1 and the planes in flight; the march is unrolled by
// NS so the rotation is a renaming, not a copy, and a set is reloaded only
// after its last use (each wait is then for the oldest plane in flight).
template <typename T, int MODE, int OP, int PF, int WPE, int SH>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE))) void k_march(
    LevelView<T> L, const T *__restrict__ u, const T *__restrict__ f, T *__restrict__ y,
    double *__restrict__ partial, ChebArgs<T> cb)
{
    constexpr int NS = PF + 3;
    const int per_tet = L.vpt + L.bpt2;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    double sq = 0.0;
    if (lb < L.n_tet * per_tet) {
        const int tet = lb / per_tet;
        int bi;
        const bool marching = march_block(lb - tet * per_tet, L.vpt, L.bpt2, bi);
        const int64_t base = (int64_t)tet * L.Spad;
        if (marching) {
            const int item = __builtin_amdgcn_readfirstlane(bi * 4 + (threadIdx.x >> 6));
            if (item < L.n_items) {
                const uint2 it = L.items[item];
                const int n = L.n, lane = threadIdx.x & 63;
                const int k0 = __builtin_amdgcn_readfirstlane((int)(it.y & 0xffffu));
                const int k1 = __builtin_amdgcn_readfirstlane((int)(it.y >> 16));
                const int t = (int)it.x - 1 + lane;
                int sd = t >= 0 ? (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f) : -1;
                if (t >= 0) {
                    while ((sd + 1) * (sd + 2) / 2 <= t) ++sd;
                    while (sd > 0 && sd * (sd + 1) / 2 > t) --sd;
                }
                const int i = t - sd * (sd + 1) / 2;
                const bool row_lane = t >= 0 && lane >= 1 && lane <= 62 && i >= 1 && i <= sd - 1;
                const int kend = n - 1 - sd;  // last interior plane of this column
                constexpr int B = (int)sizeof(T);
                const __amdgpu_buffer_rsrc_t ru = tet_rsrc(u + base, (int64_t)L.S * B);
                const __amdgpu_buffer_rsrc_t rk = tet_rsrc(L.kap + base, (int64_t)L.S * B);
                const __amdgpu_buffer_rsrc_t rf = tet_rsrc(MODE != MODE_APPLY ? f + base : u + base,
                                                           (int64_t)L.S * B);
                const __amdgpu_buffer_rsrc_t rd = tet_rsrc(MODE == MODE_CHEB ? cb.d + base : u + base,
                                                           (int64_t)L.S * B);
                const __amdgpu_buffer_rsrc_t ri = tet_rsrc(MODE == MODE_CHEB ? cb.invd + base : u + base,
                                                           (int64_t)L.S * B);
                const __amdgpu_buffer_rsrc_t ry = tet_rsrc(y + base, (int64_t)L.S * B);
                // in-plane offsets of diagonals s-1, s, s+1 at position i (a
                // lane left of the tet's first column reads offset 0: in range
                // and unused)
                const int vo[3] = {t >= 0 ? t - sd : 0, t >= 0 ? t : 0, t >= 0 ? t + sd + 1 : 0};
                const int Sn = tc32(n);
                // first slot of plane p; for planes past the top (p <= n + 2NS)
                // this is >= Sn, so their slots lie beyond the tet's range
                auto plane = [&](int p) { return Sn - tc32(n - p); };
                T wr[NDIR / 2];
                const T *__restrict__ w = OP == 0 ? L.sten + (int64_t)tet * TET_STENCIL
                                                  : L.emat + (int64_t)tet * TET_EMAT;
                if (OP == 0) {
#pragma unroll
                    for (int d = 0; d < NDIR / 2; ++d) wr[d] = w[d];
                }
                MPlane<T> R[NS];
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    mplane_load<T, MODE>(R[q], ru, rk, rf, rd, ri, vo, plane(k0 - 1 + q));
                    // keep the sets in issue order (waits go by issue order)
                    __builtin_amdgcn_sched_barrier(0);
                }
                mplane_shift_mid(R[0]);
                mplane_shift_up(R[1]);
                // the unrolled body has no branch: every lane computes, and a
                // lane without a row at this plane (or a step past the chunk)
                // stores to a byte offset beyond the tet's range, which the
                // buffer range check drops.  The wait for a plane's loads is
                // then the same at every step.
                const int lastk = row_lane ? min(kend, k1) : -1;
                constexpr int DROP = 0x7ffffff0;
                for (int kb = k0; kb <= k1; kb += NS) {
#pragma unroll
                    for (int q = 0; q < NS; ++q) {
                        const int k = kb + q;
                        MPlane<T> &M = R[q % NS], &C = R[(q + 1) % NS], &P = R[(q + 2) % NS];
                        if (SH) {
                            mplane_renew(M);
                            mplane_renew(C);
                            mplane_renew(P);
                            mplane_shift_mid(M);
                            mplane_shift_up(C);
                        }
                        mplane_shift_mid(C);
                        mplane_shift_up(P);
                        // neighbours in DIR order, centre last
                        const T uu[NDIR + 1] = {C.u_sp_r, C.u[2], P.u[1], C.u_s_r, M.u_sp_r, M.u[2],
                                                P.u_s_r, C.u_sm_l, C.u[0], M.u[1], C.u_s_l, P.u_sm_l,
                                                P.u[0], M.u_s_l, C.u[1]};
                        const T kk[NDIR + 1] = {C.k_sp_r, C.k[2], P.k[1], C.k_s_r, M.k_sp_r, M.k[2],
                                                P.k_s_r, C.k_sm_l, C.k[0], M.k[1], C.k_s_l, P.k_sm_l,
                                                P.k[0], M.k_s_l, C.k[1]};
                        const T acc = OP == 0 ? scaled_row_paired<T>(uu, kk, wr) : row_value<T, OP>(uu, kk, w);
                        const bool live = k <= lastk;
                        const int so = live ? (plane(k) + vo[1]) * B : DROP;
                        if (MODE == MODE_APPLY) {
                            bstore(acc, ry, so);
                        } else if (MODE == MODE_RESID) {
                            const T r = C.f - acc;
                            bstore(r, ry, so);
                            sq += live ? (double)r * (double)r : 0.0;
                        } else {
                            const T r = C.f - acc;
                            const T dn = (cb.first ? T(0) : cb.c_old * C.d) + cb.c_r * C.id * r;
                            bstore(dn, rd, so);
                            bstore(C.u[1] + dn, ry, so);
                        }
                        // plane k-1 is done with: its set takes plane k-1+NS
                        mplane_load<T, MODE>(M, ru, rk, rf, rd, ri, vo, plane(k - 1 + NS));
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
        } else {
            const int e = bi * BLOCK + threadIdx.x;
            if (e < L.n_bnd) {
                const uint32_t v = L.bnd[e];
                if ((L.dmask[tet] >> (v & 15u)) & 1) y[base + (v >> 4)] = T(0);
            }
        }
    }
    if (MODE == MODE_RESID) {
        sq = block_reduce(sq, 0);
        if (threadIdx.x == 0) partial[blockIdx.x] = sq;
    }
}


// ---------------------------------------------------------------- two rows per lane
// The same column march with each lane holding two consecutive in-plane
// offsets (x = t0 - 1 + 2 lane, y = x + 1), so one 16-byte (FP64) or 8-byte
// (FP32) load per anti-diagonal serves two rows and a wave produces 126 rows
// per plane (x of lane 0 and y of lane 63 only feed their neighbours).  Left
// neighbours of y and right neighbours of x are in the lane itself; the
// others come from the adjacent lanes.  Loads of diagonal s-1 start at y's
// offset and those of s+1 at x's: when a lane straddles two diagonals (x the
// last node of diagonal s, y the first of s+1) the pair then still holds the
// value each element's row neighbours use (x's s-1 and y's s+1 values are
// used by no row in that case).
template <typename T>
struct P2 {
    T x, y;
};
template <typename T>
__device__ __forceinline__ P2<T> bload2(__amdgpu_buffer_rsrc_t r, int idx);
template <>
__device__ __forceinline__ P2<double> bload2<double>(__amdgpu_buffer_rsrc_t r, int idx)
{
    const auto q = __builtin_amdgcn_raw_buffer_load_b128(r, idx * 8, 0, 0);
    P2<double> v;
    __builtin_memcpy(&v, &q, 16);
    return v;
}
template <>
__device__ __forceinline__ P2<float> bload2<float>(__amdgpu_buffer_rsrc_t r, int idx)
{
    const auto q = __builtin_amdgcn_raw_buffer_load_b64(r, idx * 4, 0, 0);
    P2<float> v;
    __builtin_memcpy(&v, &q, 8);
    return v;
}

template <typename T>
struct MPlane2 {
    P2<T> u[3], k[3], f, d, id;
};

template <typename T, int MODE>
__device__ __forceinline__ void mplane2_load(MPlane2<T> &p, __amdgpu_buffer_rsrc_t ru, __amdgpu_buffer_rsrc_t rk,
                                             __amdgpu_buffer_rsrc_t rf, __amdgpu_buffer_rsrc_t rd,
                                             __amdgpu_buffer_rsrc_t ri, const int o[3], int P)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) p.u[c] = bload2<T>(ru, P + o[c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) p.k[c] = bload2<T>(rk, P + o[c]);
    if (MODE != MODE_APPLY) p.f = bload2<T>(rf, P + o[1]);
    if (MODE == MODE_CHEB) {
        p.d = bload2<T>(rd, P + o[1]);
        p.id = bload2<T>(ri, P + o[1]);
    }
}

// the 15 values of x's and y's rows for one array: planes M (k-1), C (k), P (k+1)
template <typename T>
__device__ __forceinline__ void gather2(const P2<T> *M, const P2<T> *C, const P2<T> *P, T vx[NDIR + 1],
                                        T vy[NDIR + 1])
{
    // lane shifts: left of x = y of lane-1, right of y = x of lane+1
    const T C_sm_lx = dpp_prev(C[0].y), C_s_lx = dpp_prev(C[1].y);
    const T C_s_ry = dpp_next(C[1].x), C_sp_ry = dpp_next(C[2].x);
    const T P_sm_lx = dpp_prev(P[0].y), P_s_ry = dpp_next(P[1].x);
    const T M_sp_ry = dpp_next(M[2].x), M_s_lx = dpp_prev(M[1].y);
    // DIR order: (1,0,0) (0,1,0) (0,0,1) (1,-1,0) (1,0,-1) (0,1,-1) (1,-1,1), negatives, centre
    vx[0] = C[2].y;  vy[0] = C_sp_ry;   // s+1, i+1
    vx[1] = C[2].x;  vy[1] = C[2].y;    // s+1, i
    vx[2] = P[1].x;  vy[2] = P[1].y;    // plane k+1: s, i
    vx[3] = C[1].y;  vy[3] = C_s_ry;    // s, i+1
    vx[4] = M[2].y;  vy[4] = M_sp_ry;   // plane k-1: s+1, i+1
    vx[5] = M[2].x;  vy[5] = M[2].y;    // plane k-1: s+1, i
    vx[6] = P[1].y;  vy[6] = P_s_ry;    // plane k+1: s, i+1
    vx[7] = C_sm_lx; vy[7] = C[0].x;    // s-1, i-1
    vx[8] = C[0].x;  vy[8] = C[0].y;    // s-1, i
    vx[9] = M[1].x;  vy[9] = M[1].y;    // plane k-1: s, i
    vx[10] = C_s_lx; vy[10] = C[1].x;   // s, i-1
    vx[11] = P_sm_lx; vy[11] = P[0].x;  // plane k+1: s-1, i-1
    vx[12] = P[0].x; vy[12] = P[0].y;   // plane k+1: s-1, i
    vx[13] = M_s_lx; vy[13] = M[1].x;   // plane k-1: s, i-1
    vx[14] = C[1].x; vy[14] = C[1].y;   // centre
}

__device__ __forceinline__ void bstore_drop(double v, __amdgpu_buffer_rsrc_t r, int voff) { bstore(v, r, voff); }
__device__ __forceinline__ void bstore_drop(float v, __amdgpu_buffer_rsrc_t r, int voff) { bstore(v, r, voff); }

// WPB waves per block (4: BLOCK threads; 1: one wave per block)
template <int WPB>
static inline int march2_blocks_per_tet(int n_items2, int n_bnd)
{
    return (n_items2 + WPB - 1) / WPB + (n_bnd + 64 * WPB - 1) / (64 * WPB);
}

template <typename T, int MODE, int OP, int PF, int WPE, int WPB = 4>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(WPE))) void k_march2(
    LevelView<T> L, const T *__restrict__ u, const T *__restrict__ f, T *__restrict__ y,
    double *__restrict__ partial, ChebArgs<T> cb)
{
    constexpr int NS = PF + 3;
    const int vb = (L.n_items2 + WPB - 1) / WPB;
    const int per_tet = vb + (L.n_bnd + 64 * WPB - 1) / (64 * WPB);
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    double sq = 0.0;
    if (lb < L.n_tet * per_tet) {
        const int tet = lb / per_tet;
        int bi;
        const bool marching = march_block(lb - tet * per_tet, vb, per_tet - vb, bi);
        const int64_t base = (int64_t)tet * L.Spad;
        if (marching) {
            const int item = __builtin_amdgcn_readfirstlane(bi * WPB + (threadIdx.x >> 6));
            if (item < L.n_items2) {
                const uint2 it = L.items2[item];
                const int n = L.n, lane = threadIdx.x & 63;
                const int k0 = __builtin_amdgcn_readfirstlane((int)(it.y & 0xffffu));
                const int k1 = __builtin_amdgcn_readfirstlane((int)(it.y >> 16));
                const int tx = (int)it.x - 1 + 2 * lane, ty = tx + 1;
                auto diag = [](int t) {
                    int d = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
                    while ((d + 1) * (d + 2) / 2 <= t) ++d;
                    while (d > 0 && d * (d + 1) / 2 > t) --d;
                    return d;
                };
                const int sdx = tx >= 0 ? diag(tx) : -1, sdy = diag(ty);
                const int ix = tx - sdx * (sdx + 1) / 2, iy = ty - sdy * (sdy + 1) / 2;
                const bool row_x = tx >= 0 && lane >= 1 && ix >= 1 && ix <= sdx - 1;
                const bool row_y = lane <= 62 && iy >= 1 && iy <= sdy - 1;
                const int lastx = row_x ? min(n - 1 - sdx, k1) : -1;
                const int lasty = row_y ? min(n - 1 - sdy, k1) : -1;
                constexpr int B = (int)sizeof(T);
                const __amdgpu_buffer_rsrc_t ru = tet_rsrc(u + base, (int64_t)L.S * B);
                const __amdgpu_buffer_rsrc_t rk = tet_rsrc(L.kap + base, (int64_t)L.S * B);
                const __amdgpu_buffer_rsrc_t rf = tet_rsrc(MODE != MODE_APPLY ? f + base : u + base,
                                                           (int64_t)L.S * B);
                const __amdgpu_buffer_rsrc_t rd = tet_rsrc(MODE == MODE_CHEB ? cb.d + base : u + base,
                                                           (int64_t)L.S * B);
                const __amdgpu_buffer_rsrc_t ri = tet_rsrc(MODE == MODE_CHEB ? cb.invd + base : u + base,
                                                           (int64_t)L.S * B);
                const __amdgpu_buffer_rsrc_t ry = tet_rsrc(y + base, (int64_t)L.S * B);
                // pair start offsets of diagonals s-1 (from y), s, s+1 (from x); a
                // negative start (left of the tet's first column) reads offset 0
                const int osm = ty - sdy - 1, oc = tx, osp = tx + sdx + 1;
                const int vo[3] = {osm >= 0 ? osm : 0, oc >= 0 ? oc : 0, osp >= 0 ? osp : 0};
                const int Sn = tc32(n);
                auto plane = [&](int p) { return Sn - tc32(n - p); };
                T wr[NDIR / 2];
                const T *__restrict__ w = OP == 0 ? L.sten + (int64_t)tet * TET_STENCIL
                                                  : L.emat + (int64_t)tet * TET_EMAT;
                if (OP == 0) {
#pragma unroll
                    for (int d = 0; d < NDIR / 2; ++d) wr[d] = w[d];
                }
                MPlane2<T> R[NS];
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    mplane2_load<T, MODE>(R[q], ru, rk, rf, rd, ri, vo, plane(k0 - 1 + q));
                    __builtin_amdgcn_sched_barrier(0);
                }
                constexpr int DROP = 0x7ffffff0;
                for (int kb = k0; kb <= k1; kb += NS) {
#pragma unroll
                    for (int q = 0; q < NS; ++q) {
                        const int k = kb + q;
                        MPlane2<T> &M = R[q % NS], &C = R[(q + 1) % NS], &P = R[(q + 2) % NS];
                        T ux[NDIR + 1], uy[NDIR + 1], kx[NDIR + 1], ky[NDIR + 1];
                        gather2<T>(M.u, C.u, P.u, ux, uy);
                        gather2<T>(M.k, C.k, P.k, kx, ky);
                        const T ax = OP == 0 ? scaled_row_paired<T>(ux, kx, wr) : row_value<T, OP>(ux, kx, w);
                        const T ay = OP == 0 ? scaled_row_paired<T>(uy, ky, wr) : row_value<T, OP>(uy, ky, w);
                        const int Pk = plane(k);
                        const bool lx = k <= lastx, ly = k <= lasty;
                        const int sx = lx ? (Pk + tx) * B : DROP, sy = ly ? (Pk + ty) * B : DROP;
                        if (MODE == MODE_APPLY) {
                            bstore(ax, ry, sx);
                            bstore(ay, ry, sy);
                        } else if (MODE == MODE_RESID) {
                            const T rx = C.f.x - ax, rv = C.f.y - ay;
                            bstore(rx, ry, sx);
                            bstore(rv, ry, sy);
                            sq += (lx ? (double)rx * (double)rx : 0.0) + (ly ? (double)rv * (double)rv : 0.0);
                        } else {
                            const T rx = C.f.x - ax, rv = C.f.y - ay;
                            const T dx = (cb.first ? T(0) : cb.c_old * C.d.x) + cb.c_r * C.id.x * rx;
                            const T dy = (cb.first ? T(0) : cb.c_old * C.d.y) + cb.c_r * C.id.y * rv;
                            bstore(dx, rd, sx);
                            bstore(dy, rd, sy);
                            bstore(C.u[1].x + dx, ry, sx);
                            bstore(C.u[1].y + dy, ry, sy);
                        }
                        mplane2_load<T, MODE>(M, ru, rk, rf, rd, ri, vo, plane(k - 1 + NS));
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
        } else {
            const int e = bi * (64 * WPB) + threadIdx.x;
            if (e < L.n_bnd) {
                const uint32_t v = L.bnd[e];
                if ((L.dmask[tet] >> (v & 15u)) & 1) y[base + (v >> 4)] = T(0);
            }
        }
    }
    if (MODE == MODE_RESID) {
        if (WPB == 4) sq = block_reduce(sq, 0);
        else sq = warp_sum(sq);
        if (threadIdx.x == 0) partial[blockIdx.x] = sq;
    }
}

// ---------------------------------------------------------------- LDS-staged block march
// Eight waves march 1008 consecutive offsets of a plane chunk together (each
// wave two rows per lane as in k_march2).  Per plane the block copies the
// region of offsets its rows touch (at most 1536 elements per array) straight
// from HBM into an LDS ring with 16-byte-per-lane buffer-to-LDS loads, so
// every value of the plane is fetched once per block instead of once per
// diagonal and wave; each wave then reads its three diagonal pairs per array
// from LDS.  Two planes are in flight; one barrier per plane orders the ring.
// The LDS reads are written as inline asm that waits for its own data, and the
// waits for the LDS loads are explicit (counted per wave): the compiler would
// otherwise wait for every outstanding load before each LDS read.
// FP64: a 16-byte load brings 2 elements per lane, 128 per wave and load:
// twelve chunks per array, three loads per wave and plane.  FP32: 4 elements
// per lane, 256 per load: six chunks per array, two load slots per wave and
// plane (16 slots for 12 chunks; the spare slots read nothing).
constexpr int LW = 8;               // waves per block
constexpr int LELEM = 1536;         // staged elements per array and plane
constexpr int LRS = 3;              // ring slots (two planes in flight)

template <typename T>
struct LdsCfg;
template <>
struct LdsCfg<double> {
    static constexpr int CHUNK = 128;  // elements per 16-byte-per-lane load
    static constexpr int LCH = LELEM / CHUNK;
    static constexpr int PERWAVE = 3;  // load slots per wave and plane
};
template <>
struct LdsCfg<float> {
    static constexpr int CHUNK = 256;
    static constexpr int LCH = LELEM / CHUNK;
    static constexpr int PERWAVE = 2;
};

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ unsigned lds_addr(const T *p)
{
    return (unsigned)(size_t)((__attribute__((address_space(3))) const T *)p);
}

// the six pairs (diagonals s-1, s, s+1 of u and k) of one plane from LDS
__device__ __forceinline__ void lds_read_plane(unsigned au, unsigned ak, const int e[3], P2<double> uu[3],
                                               P2<double> kk[3])
{
    d2v a0, a1, a2, b0, b1, b2;
    asm volatile(
        "ds_read2_b64 %0, %6 offset1:1\n\t"
        "ds_read2_b64 %1, %7 offset1:1\n\t"
        "ds_read2_b64 %2, %8 offset1:1\n\t"
        "ds_read2_b64 %3, %9 offset1:1\n\t"
        "ds_read2_b64 %4, %10 offset1:1\n\t"
        "ds_read2_b64 %5, %11 offset1:1\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(b0), "=&v"(b1), "=&v"(b2)
        : "v"(au + e[0] * 8), "v"(au + e[1] * 8), "v"(au + e[2] * 8), "v"(ak + e[0] * 8), "v"(ak + e[1] * 8),
          "v"(ak + e[2] * 8)
        : "memory");
    uu[0] = {a0.x, a0.y}; uu[1] = {a1.x, a1.y}; uu[2] = {a2.x, a2.y};
    kk[0] = {b0.x, b0.y}; kk[1] = {b1.x, b1.y}; kk[2] = {b2.x, b2.y};
}
__device__ __forceinline__ void lds_read_plane(unsigned au, unsigned ak, const int e[3], P2<float> uu[3],
                                               P2<float> kk[3])
{
    f2v a0, a1, a2, b0, b1, b2;
    asm volatile(
        "ds_read2_b32 %0, %6 offset1:1\n\t"
        "ds_read2_b32 %1, %7 offset1:1\n\t"
        "ds_read2_b32 %2, %8 offset1:1\n\t"
        "ds_read2_b32 %3, %9 offset1:1\n\t"
        "ds_read2_b32 %4, %10 offset1:1\n\t"
        "ds_read2_b32 %5, %11 offset1:1\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(b0), "=&v"(b1), "=&v"(b2)
        : "v"(au + e[0] * 4), "v"(au + e[1] * 4), "v"(au + e[2] * 4), "v"(ak + e[0] * 4), "v"(ak + e[1] * 4),
          "v"(ak + e[2] * 4)
        : "memory");
    uu[0] = {a0.x, a0.y}; uu[1] = {a1.x, a1.y}; uu[2] = {a2.x, a2.y};
    kk[0] = {b0.x, b0.y}; kk[1] = {b1.x, b1.y}; kk[2] = {b2.x, b2.y};
}

// s_waitcnt immediates (gfx9 encoding: vmcnt in bits 3:0, expcnt 6:4 (7 = no
// wait), lgkmcnt 11:8 (15 = no wait)) for vmcnt(n), n < 16
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 16, "vmcnt immediate");
    __builtin_amdgcn_s_waitcnt(0x0F70 | N);
}

// row values of one plane (two rows per lane): f, and for the smoother the
// direction d and D^-1 at x and y
template <typename T>
struct LdsRow {
    P2<T> f, d, id;
};

// one 16-byte (FP64) or 8-byte (FP32) load of a lane's two row values
template <typename T>
__device__ __forceinline__ P2<T> load_pair(__amdgpu_buffer_rsrc_t r, int off)
{
    if constexpr (sizeof(T) == 8) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
        unsigned long long lo = ((unsigned long long)v[1] << 32) | v[0], hi = ((unsigned long long)v[3] << 32) | v[2];
        P2<T> o;
        __builtin_memcpy(&o.x, &lo, 8);
        __builtin_memcpy(&o.y, &hi, 8);
        return o;
    } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        return {__uint_as_float(v[0]), __uint_as_float(v[1])};
    }
}

// block sum of an 8-wave block, the result in thread 0
__device__ __forceinline__ double block_reduce_lw(double v)
{
    __shared__ double red[LW];
    v = warp_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 1; q < LW; ++q) v += red[q];
    return v;
}

template <typename T, int MODE>
__global__ __launch_bounds__(64 * LW) __attribute__((amdgpu_waves_per_eu(4))) void k_march_lds(
    LevelView<T> L, const T *__restrict__ u, const T *__restrict__ f, T *__restrict__ y,
    double *__restrict__ partial, ChebArgs<T> cb)
{
    using C = LdsCfg<T>;
    constexpr int B = (int)sizeof(T);
    // row loads per plane (f; f, d, D^-1) and stores per step (y; d, u_new)
    constexpr int RL = MODE == MODE_APPLY ? 0 : MODE == MODE_RESID ? 1 : 3;
    constexpr int ST = MODE == MODE_CHEB ? 4 : 2;
    __shared__ __attribute__((aligned(16))) T ring[LRS][2][LELEM];
    // landing area of the spare load slots (FP32): they read nothing, and
    // whatever the hardware writes for them must not reach the ring
    __shared__ __attribute__((aligned(16))) T dump[64 * 16 / sizeof(T)];
    const int nbb = (L.n_bnd + 64 * LW - 1) / (64 * LW);
    const int per_tet = L.n_itemsL + nbb;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    if (lb >= L.n_tet * per_tet) {  // whole block
        if (MODE == MODE_RESID && threadIdx.x == 0) partial[blockIdx.x] = 0.0;
        return;
    }
    const int tet = lb / per_tet;
    int b;
    const bool marching = march_block(lb - tet * per_tet, L.n_itemsL, nbb, b);
    const int64_t base = (int64_t)tet * L.Spad;
    if (!marching) {  // whole block: Dirichlet zeros
        const int e = b * (64 * LW) + threadIdx.x;
        if (e < L.n_bnd) {
            const uint32_t v = L.bnd[e];
            if ((L.dmask[tet] >> (v & 15u)) & 1) y[base + (v >> 4)] = T(0);
        }
        if (MODE == MODE_RESID && threadIdx.x == 0) partial[blockIdx.x] = 0.0;
        return;
    }
    const uint2 it = L.itemsL[b];
    const int n = L.n;
    const int t0 = __builtin_amdgcn_readfirstlane((int)it.x);
    const int k0 = __builtin_amdgcn_readfirstlane((int)(it.y & 0xffffu));
    const int k1 = __builtin_amdgcn_readfirstlane((int)(it.y >> 16));
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    auto diag = [](int t) {
        int d = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while ((d + 1) * (d + 2) / 2 <= t) ++d;
        while (d > 0 && d * (d + 1) / 2 > t) --d;
        return d;
    };
    const int tx = t0 - 1 + 126 * wave + 2 * lane, ty = tx + 1;
    const int sdx = tx >= 0 ? diag(tx) : -1, sdy = diag(ty);
    const int ix = tx - sdx * (sdx + 1) / 2, iy = ty - sdy * (sdy + 1) / 2;
    const bool row_x = tx >= 0 && lane >= 1 && ix >= 1 && ix <= sdx - 1;
    const bool row_y = lane <= 62 && iy >= 1 && iy <= sdy - 1;
    const int lastx = row_x ? min(n - 1 - sdx, k1) : -1;
    const int lasty = row_y ? min(n - 1 - sdy, k1) : -1;
    // staged region of every plane: in-plane offsets [lo, lo + need), need <=
    // LELEM: from diagonal s-1 of the first row to diagonal s+1 of the last
    // (x of the last lane of the last wave sits at t0 + 1007)
    const int lo = __builtin_amdgcn_readfirstlane(t0 - diag(t0) - 1);
    const int need = __builtin_amdgcn_readfirstlane(t0 + 1007 + diag(t0 + 1007) + 3 - lo);
    const int osm = ty - sdy - 1, oc = tx, osp = tx + sdx + 1;
    const int e[3] = {(osm >= 0 ? osm : 0) - lo, (oc >= 0 ? oc : 0) - lo, (osp >= 0 ? osp : 0) - lo};
    const __amdgpu_buffer_rsrc_t ru = tet_rsrc(u + base, (int64_t)L.S * B);
    const __amdgpu_buffer_rsrc_t rk = tet_rsrc(L.kap + base, (int64_t)L.S * B);
    const __amdgpu_buffer_rsrc_t ry = tet_rsrc(y + base, (int64_t)L.S * B);
    const __amdgpu_buffer_rsrc_t rf = tet_rsrc(MODE != MODE_APPLY ? f + base : u + base, (int64_t)L.S * B);
    const __amdgpu_buffer_rsrc_t rd = tet_rsrc(MODE == MODE_CHEB ? cb.d + base : u + base, (int64_t)L.S * B);
    const __amdgpu_buffer_rsrc_t ri = tet_rsrc(MODE == MODE_CHEB ? cb.invd + base : u + base, (int64_t)L.S * B);
    const int Sn = tc32(n);
    auto plane = [&](int p) { return Sn - tc32(n - p); };
    constexpr int DROP = 0x7ffffff0;
    // this wave's 16-byte-per-lane LDS loads of plane p into slot p % LRS
    auto stage = [&](int p) {
        const int sl = p % LRS;
#pragma unroll
        for (int q = 0; q < C::PERWAVE; ++q) {
            const int Q = wave * C::PERWAVE + q;
            const int arr = Q / C::LCH, ch = Q - arr * C::LCH;
            // a chunk past the needed length, or a plane past the last one
            // the chunk's rows use, is still issued (the waits count
            // PERWAVE loads per wave and plane) but reads nothing and lands
            // in its own chunk, which no row reads; a spare slot past the
            // two arrays' chunks lands in the dump area
            const bool spare = arr >= 2;
            const bool real = !spare && ch * C::CHUNK < need && p <= k1 + 1;
            const int voff = real ? (plane(p) + lo + ch * C::CHUNK + (16 / B) * lane) * B : DROP;
            T *dst = spare ? &dump[0] : &ring[sl][spare ? 0 : arr][spare ? 0 : ch * C::CHUNK];
            __builtin_amdgcn_raw_ptr_buffer_load_lds(arr == 1 ? rk : ru, (__attribute__((address_space(3))) void *)dst,
                                                     16, voff, 0, 0, 0);
        }
    };
    // the row values of plane p (RL loads; a plane without a row reads nothing)
    auto rowload = [&](int p, LdsRow<T> &v) {
        if constexpr (RL > 0) {
            const int off = (p <= lastx || p <= lasty) ? (plane(p) + tx) * B : DROP;
            v.f = load_pair<T>(rf, off);
            if constexpr (RL == 3) {
                v.d = load_pair<T>(rd, off);
                v.id = load_pair<T>(ri, off);
            }
        }
    };
    auto addr = [&](int p, int arr) { return lds_addr<T>(&ring[p % LRS][arr][0]); };
    T wr[NDIR / 2];
    const T *__restrict__ w = L.sten + (int64_t)tet * TET_STENCIL;
#pragma unroll
    for (int d = 0; d < NDIR / 2; ++d) wr[d] = w[d];
    struct Pl {
        P2<T> u[3], k[3];
    } R[3];
    LdsRow<T> RV[3];
    double sq = 0.0;
    // prologue: planes k0-1 and k0 into registers, then k0+1 and k0+2 in
    // flight, then the row values of plane k0
    stage(k0 - 1);
    stage(k0);
    __builtin_amdgcn_sched_barrier(0);
    wait_vm<0>();
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    lds_read_plane(addr(k0 - 1, 0), addr(k0 - 1, 1), e, R[0].u, R[0].k);
    lds_read_plane(addr(k0, 0), addr(k0, 1), e, R[1].u, R[1].k);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    stage(k0 + 1);
    stage(k0 + 2);
    rowload(k0, RV[0]);
    __builtin_amdgcn_sched_barrier(0);
    for (int kb = k0; kb <= k1; kb += 3) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int k = kb + q;
            if (k > k1) break;  // block-uniform
            Pl &M = R[q % 3], &Cc = R[(q + 1) % 3], &P = R[(q + 2) % 3];
            const LdsRow<T> &rv = RV[q % 3];
            // plane k+1 has landed once at most the later loads and stores
            // are outstanding: at the first step the next plane's PERWAVE
            // loads and this plane's row loads; later the previous step's row
            // loads (of this plane), stores and plane loads, issued in that
            // order
            __builtin_amdgcn_sched_barrier(0);
            if (k == k0) wait_vm<C::PERWAVE + RL>();
            else wait_vm<RL + ST + C::PERWAVE>();
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_sched_barrier(0);
            lds_read_plane(addr(k + 1, 0), addr(k + 1, 1), e, P.u, P.k);
            T ux[NDIR + 1], uy[NDIR + 1], kx[NDIR + 1], ky[NDIR + 1];
            gather2<T>(M.u, Cc.u, P.u, ux, uy);
            gather2<T>(M.k, Cc.k, P.k, kx, ky);
            const T ax = scaled_row_paired<T>(ux, kx, wr);
            const T ay = scaled_row_paired<T>(uy, ky, wr);
            const int Pk = plane(k);
            const bool lx = k <= lastx, ly = k <= lasty;
            const int sx = lx ? (Pk + tx) * B : DROP, sy = ly ? (Pk + ty) * B : DROP;
            // the next plane's row values, before this step's stores
            rowload(k + 1, RV[(q + 1) % 3]);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (MODE == MODE_APPLY) {
                bstore(ax, ry, sx);
                bstore(ay, ry, sy);
            } else if constexpr (MODE == MODE_RESID) {
                const T rx = rv.f.x - ax, rr = rv.f.y - ay;
                bstore(rx, ry, sx);
                bstore(rr, ry, sy);
                sq += (lx ? (double)rx * (double)rx : 0.0) + (ly ? (double)rr * (double)rr : 0.0);
            } else {
                const T rx = rv.f.x - ax, rr = rv.f.y - ay;
                const T dx = (cb.first ? T(0) : cb.c_old * rv.d.x) + cb.c_r * rv.id.x * rx;
                const T dy = (cb.first ? T(0) : cb.c_old * rv.d.y) + cb.c_r * rv.id.y * rr;
                bstore(dx, rd, sx);
                bstore(dy, rd, sy);
                bstore(Cc.u[1].x + dx, ry, sx);
                bstore(Cc.u[1].y + dy, ry, sy);
            }
            // the slot of plane k (read one step ago by every wave, which all
            // passed this step's barrier) takes plane k+3
            __builtin_amdgcn_sched_barrier(0);
            stage(k + 3);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // drain: every LDS load has landed before the block's LDS is released
    wait_vm<0>();
    if constexpr (MODE == MODE_RESID) {
        sq = block_reduce_lw(sq);
        if (threadIdx.x == 0) partial[blockIdx.x] = sq;
    }
}

template <typename T>
static int lds_grid(const LevelView<T> &L)
{
    const int nbb = (L.n_bnd + 64 * LW - 1) / (64 * LW);
    return ((L.n_tet * (L.n_itemsL + nbb) + 7) / 8) * 8;
}

static inline int march_grid(int n_tet, int vpt, int bpt2)
{
    const int nb = n_tet * (vpt + bpt2);
    return ((nb + 7) / 8) * 8;
}

// variant of the marching kernels (rows per lane, prefetch depth, occupancy,
// LDS staging): 0 = the default policy; the initial value comes from
// HHG_MARCH_VARIANT, hhg_set_kernel_variant changes it (tuning and tests)
static int g_variant = -1;
static int march_variant()
{
    if (g_variant < 0) {
        const char *e = getenv("HHG_MARCH_VARIANT");
        int v = e ? atoi(e) : 0;
        if (v < 0 || v > 10) v = 0;
        g_variant = v;
    }
    return g_variant;
}
int march_variant_now() { return march_variant(); }
int set_march_variant(int v)
{
    if (v < 0 || v > 10) return -1;
    g_variant = v;
    return 0;
}

// Timed applies (instrumentation of hhg_apply_scaled): while events are set,
// the launches of launch_march_std and launch_shared_rows go through
// hipExtLaunchKernel, which takes the start time from the first kernel's own
// dispatch and the stop time from the completion of each kernel it is given
// (the last one's counts), so the pair spans the apply's kernels and no
// separate event command.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
static thread_local LaunchEvents t_launch_ev;
void set_launch_events(hipEvent_t start, hipEvent_t stop) { t_launch_ev = LaunchEvents{start, stop}; }
bool launch_events_unused() { return t_launch_ev.start != nullptr; }

template <typename... P, typename... A>
static void launch_k(void (*kernel)(P...), dim3 grid, dim3 block, hipStream_t st, const A &...args)
{
    if (t_launch_ev.stop) {
        hipExtLaunchKernelGGL(kernel, grid, block, 0, st, t_launch_ev.start, t_launch_ev.stop, 0, args...);
        t_launch_ev.start = nullptr;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
    }
}

// scaled rows: variants 6, 8, 9 run two rows per lane, 1-5 and 7 one per
// lane; the default (0) runs FP64 two per lane and FP32 one per lane with
// shifts recomputed at each use (variant 1), the fastest of each measured
template <typename T>
static inline bool two_rows(int v) { return v == 6 || v == 8 || v == 9 || (v == 0 && sizeof(T) == 8); }

// the LDS-staged block march where the level fits it: forced by variant 10,
// chosen by default for working sets far beyond the last-level cache (it
// measured faster there and slower below; on the 48-tet cube at level 8 the
// FP64 apply 131 vs 122, the FP32 apply 205 vs 184 GDoF/s).  Residual and
// smoother sweeps use it in FP32 (the FP64 kernel's registers hold no row
// values beyond the apply's) from 8M slots on, where their five arrays no
// longer fit the last-level cache (the 6-tet cube at level 8, 17M slots:
// FP32-in-FP64 solves 8% faster).
template <typename T, int MODE>
static bool use_lds(const LevelView<T> &L)
{
    if (L.n_itemsL <= 0) return false;
    if (MODE != MODE_APPLY && sizeof(T) == 8) return false;
    const int v = march_variant();
    const bool big_set = (int64_t)L.n_tet * L.Spad >= ((int64_t)(MODE == MODE_APPLY ? 32 : 8) << 20);
    return v == 10 || (v == 0 && big_set);
}

// blocks of the interior launch (one partial sum each in residual mode)
template <typename T>
static int march_blocks(const LevelView<T> &L)
{
    if (use_lds<T, MODE_RESID>(L)) return lds_grid(L);
    const int v = march_variant();
    if (v == 9) return ((L.n_tet * march2_blocks_per_tet<1>(L.n_items2, L.n_bnd) + 7) / 8) * 8;
    return two_rows<T>(v) ? march_grid(L.n_tet, L.vpt2, L.bpt2) : march_grid(L.n_tet, L.vpt, L.bpt2);
}
// the nodal rows keep the one-row-per-lane kernel (their element sums need
// too many registers for two rows per lane)

template <typename T, int MODE, int OP>
static void launch_march_std(const LevelView<T> &L, const T *u, const T *f, T *y, double *partial,
                             hipStream_t st, const ChebArgs<T> &cb);

template <typename T, int MODE, int OP>
static void launch_march(const LevelView<T> &L, const T *u, const T *f, T *y, double *partial,
                         hipStream_t st, const ChebArgs<T> &cb = ChebArgs<T>())
{
    if constexpr (MODE == MODE_CHEB) {
        // the fused smoother sweep: FP64 two rows per lane (variant 6: no
        // plane in flight, fewer registers), FP32 one row per lane
        if constexpr (sizeof(T) == 8) {
            const int g2 = march_grid(L.n_tet, L.vpt2, L.bpt2);
            if (march_variant() == 6) k_march2<T, MODE_CHEB, 0, 0, 3><<<g2, BLOCK, 0, st>>>(L, u, f, y, partial, cb);
            else k_march2<T, MODE_CHEB, 0, 1, 2><<<g2, BLOCK, 0, st>>>(L, u, f, y, partial, cb);
        } else if (use_lds<T, MODE_CHEB>(L)) {
            k_march_lds<T, MODE_CHEB><<<lds_grid(L), 64 * LW, 0, st>>>(L, u, f, y, partial, cb);
        } else {
            k_march<T, MODE_CHEB, 0, 1, 8, 1><<<march_grid(L.n_tet, L.vpt, L.bpt2), BLOCK, 0, st>>>(L, u, f, y,
                                                                                                   partial, cb);
        }
    } else {
        launch_march_std<T, MODE, OP>(L, u, f, y, partial, st, cb);
    }
}

template <typename T, int MODE, int OP>
static void launch_march_std(const LevelView<T> &L, const T *u, const T *f, T *y, double *partial,
                             hipStream_t st, const ChebArgs<T> &cb)
{
    if constexpr (OP == 0 && (MODE == MODE_APPLY || (MODE == MODE_RESID && sizeof(T) == 4))) {
        if (use_lds<T, MODE>(L)) {
            launch_k(k_march_lds<T, MODE>, lds_grid(L), 64 * LW, st, L, u, f, y, partial, cb);
            return;
        }
    }
    if constexpr (OP == 0) {
        const int v = march_variant();
        if (two_rows<T>(v)) {
            const int g2 = march_grid(L.n_tet, L.vpt2, L.bpt2);
            if (v == 6) launch_k(k_march2<T, MODE, OP, 0, 3>, g2, BLOCK, st, L, u, f, y, partial, cb);
            else if (v == 8) launch_k(k_march2<T, MODE, OP, 2, 2>, g2, BLOCK, st, L, u, f, y, partial, cb);
            else if (v == 9) {
                const int g1 = ((L.n_tet * march2_blocks_per_tet<1>(L.n_items2, L.n_bnd) + 7) / 8) * 8;
                launch_k(k_march2<T, MODE, OP, 1, 2, 1>, g1, 64, st, L, u, f, y, partial, cb);
            }
            else launch_k(k_march2<T, MODE, OP, 1, 2>, g2, BLOCK, st, L, u, f, y, partial, cb);
            return;
        }
    }
    const int g = march_grid(L.n_tet, L.vpt, L.bpt2);
    // FP64 residual and nodal rows hold more values: a lower occupancy
    // target keeps them out of scratch
    constexpr bool big = sizeof(T) == 8 && (MODE == MODE_RESID || OP == 1);
    constexpr int W4 = big ? 3 : 4;
    constexpr bool f64 = sizeof(T) == 8;
    int v = march_variant();
    if (v == 0 && OP == 0 && sizeof(T) == 4) v = 1;
    switch (v) {
    case 1: launch_k(k_march<T, MODE, OP, 1, big ? 3 : (f64 ? 5 : 8), 1>, g, BLOCK, st, L, u, f, y, partial, cb); break;
    case 2: launch_k(k_march<T, MODE, OP, 2, W4, 0>, g, BLOCK, st, L, u, f, y, partial, cb); break;
    case 3: launch_k(k_march<T, MODE, OP, 2, big ? 3 : (f64 ? 4 : 6), 1>, g, BLOCK, st, L, u, f, y, partial, cb); break;
    case 4: launch_k(k_march<T, MODE, OP, 0, 8, 1>, g, BLOCK, st, L, u, f, y, partial, cb); break;
    case 5: launch_k(k_march<T, MODE, OP, 0, big ? 5 : 6, 0>, g, BLOCK, st, L, u, f, y, partial, cb); break;
    default: launch_k(k_march<T, MODE, OP, 1, W4, 0>, g, BLOCK, st, L, u, f, y, partial, cb); break;
    }
}

// rows of nodes on primitives shared by several tets (Sec. 2.2: the row is
// the sum of the tet-restricted stencils of all copies).  The merged
// coefficients are built once per coefficient field (k_shared_coef); a row
// is then sum_m c_m (u_m - u_q), written to every copy of the node.
template <typename T, int MODE, typename IX>
__global__ __launch_bounds__(BLOCK) void k_shared_rows(LevelView<T> L, const IX *__restrict__ nbs,
                                                        const IX *__restrict__ selfs, const IX *__restrict__ cslots,
                                                        const T *__restrict__ coef, const T *__restrict__ u,
                                                        const T *__restrict__ f, T *__restrict__ y,
                                                        double *__restrict__ partial, ChebArgs<T> cb,
                                                        const T *__restrict__ coefn, int nodal_mask)
{
    const int q = blockIdx.x * BLOCK + threadIdx.x;
    const int ns = L.n_shared;
    double sq = 0.0;
    if (q < ns) {
        const int64_t self = (int64_t)selfs[q];
        const T u0 = u[self];
        // primitive-mixed operator: the nodal coefficients on the chosen primitives
        const T *__restrict__ cp = nodal_mask && (L.sh_prim[q] & nodal_mask) ? coefn : coef;
        T acc = T(0);
        for (int m = 0; m < L.sh_w; ++m) {
            const int64_t e = (int64_t)m * ns + q;
            acc += cp[e] * (u[(int64_t)nbs[e]] - u0);
        }
        T out = acc;
        if (MODE == MODE_RESID) {
            out = f[self] - acc;
            sq = (double)out * (double)out;
        }
        if (MODE == MODE_CHEB) {
            const T r = f[self] - acc;
            const T dn = (cb.first ? T(0) : cb.c_old * cb.d[self]) + cb.c_r * cb.invd[self] * r;
            cb.d[self] = dn;  // d is read at the first copy only
            for (int c = L.sh_off[q]; c < L.sh_off[q + 1]; ++c) y[(int64_t)cslots[c]] = u0 + dn;
        } else {
            for (int c = L.sh_off[q]; c < L.sh_off[q + 1]; ++c) y[(int64_t)cslots[c]] = out;
        }
    }
    if (MODE == MODE_RESID) {
        sq = block_reduce(sq, 0);
        if (threadIdx.x == 0) partial[blockIdx.x] = sq;
    }
}

// 32-bit slot lists when the level has them (and the pattern in L.sh_nb is
// the one they mirror: the tensor pattern clears sh_nb32)
template <typename T, int MODE>
static void launch_shared_rows(const LevelView<T> &L, const T *coef, const T *u, const T *f, T *y,
                               double *partial, hipStream_t st, const ChebArgs<T> &cb = ChebArgs<T>(),
                               const T *coefn = nullptr, int nodal_mask = 0)
{
    const int gs = blocks_for(L.n_shared);
    if (!gs) return;
    if (L.sh_nb32)
        launch_k(k_shared_rows<T, MODE, uint32_t>, gs, BLOCK, st, L, L.sh_nb32, L.sh_self32, L.sh_cslot32, coef, u,
                 f, y, partial, cb, coefn, nodal_mask);
    else
        launch_k(k_shared_rows<T, MODE, int64_t>, gs, BLOCK, st, L, L.sh_nb, L.sh_self, L.sh_cslot, coef, u, f, y,
                 partial, cb, coefn, nodal_mask);
}

// the scaled operator's shared rows on its own (narrower) pattern
template <typename T, int MODE>
static void launch_shared_rows_scaled(const LevelView<T> &L, const T *u, const T *f, T *y, double *partial,
                                      hipStream_t st, const ChebArgs<T> &cb = ChebArgs<T>())
{
    LevelView<T> Ls = L;
    Ls.sh_w = L.sh_ws;
    Ls.sh_nb = L.sh_nbs;
    Ls.sh_nb32 = L.sh_nbs32;
    launch_shared_rows<T, MODE>(Ls, L.sh_css, u, f, y, partial, st, cb);
}

// scaled coefficients on the scaled pattern (FP64, once per coefficient
// field): c_m = sum over copies and directions d onto m of w_d (k_q + k_m)
__global__ __launch_bounds__(BLOCK) void k_shared_coef_scaled(LevelView<double> L, const int8_t *__restrict__ map,
                                                              double *__restrict__ cs)
{
    const int q = blockIdx.x * BLOCK + threadIdx.x;
    const int ns = L.n_shared;
    if (q >= ns) return;
    for (int m = 0; m < L.sh_ws; ++m) cs[(int64_t)m * ns + q] = 0.0;
    for (int c = L.sh_off[q]; c < L.sh_off[q + 1]; ++c) {
        int tet, kind, i, j, k;
        unpack_copy(L.sh_copy[c], tet, kind, i, j, k);
        const int64_t base = (int64_t)tet * L.Spad;
        const int s = slot32(L.n, i, j, k);
        const int8_t *mp = map + (int64_t)c * 16;
        const double kq = L.kap[base + s];
        int nb[NDIR];
        neighbour_slots(s, i + j, L.n - k, nb);
        const double *w = L.sten + (int64_t)tet * TET_STENCIL + kind * KIND_STRIDE;
        for (int d = 0; d < NDIR; ++d) {
            const int m = mp[d];
            if (m >= 0) cs[(int64_t)m * ns + q] += w[d] * (kq + L.kap[base + nb[d]]);
        }
    }
}

hipError_t launch_shared_coef_scaled(const LevelView<double> &L, const int8_t *map, double *cs, hipStream_t st)
{
    if (L.n_shared) k_shared_coef_scaled<<<blocks_for(L.n_shared), BLOCK, 0, st>>>(L, map, cs);
    return hipGetLastError();
}

// merged coefficients of the shared rows (FP64, once per coefficient field):
// scaled  c_m = sum over copies and directions d onto m of w_d (k_q + k_m);
// nodal   c_m = sum over copies, elements t holding the node and m of
//         (sum of k at t's vertices) (A_t / 4)[node, m]
__global__ __launch_bounds__(BLOCK) void k_shared_coef(LevelView<double> L, const int8_t *__restrict__ map,
                                                       double *__restrict__ cs, double *__restrict__ cn)
{
    const int q = blockIdx.x * BLOCK + threadIdx.x;
    const int ns = L.n_shared;
    if (q >= ns) return;
    for (int m = 0; m < L.sh_w; ++m) {
        cs[(int64_t)m * ns + q] = 0.0;
        cn[(int64_t)m * ns + q] = 0.0;
    }
    for (int c = L.sh_off[q]; c < L.sh_off[q + 1]; ++c) {
        int tet, kind, i, j, k;
        unpack_copy(L.sh_copy[c], tet, kind, i, j, k);
        const int64_t base = (int64_t)tet * L.Spad;
        const int s = slot32(L.n, i, j, k);
        const int8_t *mp = map + (int64_t)c * 16;
        const double kq = L.kap[base + s];
        int nb[NDIR];
        neighbour_slots(s, i + j, L.n - k, nb);
        const double *w = L.sten + (int64_t)tet * TET_STENCIL + kind * KIND_STRIDE;
        for (int d = 0; d < NDIR; ++d) {
            const int m = mp[d];
            if (m >= 0) cs[(int64_t)m * ns + q] += w[d] * (kq + L.kap[base + nb[d]]);
        }
        const double *E = L.emat + (int64_t)tet * TET_EMAT;
        for (int t = 0; t < NTYPE; ++t)
            for (int a = 0; a < 4; ++a) {
                // element of shape t whose vertex a is this node
                const int bi = i - TYPE_OFF[t][a][0], bj = j - TYPE_OFF[t][a][1], bk = k - TYPE_OFF[t][a][2];
                bool ok = true;
                for (int v = 0; v < 4; ++v)
                    ok = ok && in_lattice(L.n, bi + TYPE_OFF[t][v][0], bj + TYPE_OFF[t][v][1], bk + TYPE_OFF[t][v][2]);
                if (!ok) continue;
                double ks = 0.0;
                for (int v = 0; v < 4; ++v)
                    ks += L.kap[base + slot32(L.n, bi + TYPE_OFF[t][v][0], bj + TYPE_OFF[t][v][1],
                                               bk + TYPE_OFF[t][v][2])];
                for (int v = 0; v < 4; ++v) {
                    if (v == a) continue;
                    const int m = mp[ELEM_DIR.v[t][a][v]];
                    if (m >= 0) cn[(int64_t)m * ns + q] += ks * E[t * 16 + a * 4 + v];
                }
            }
    }
}

hipError_t launch_shared_coef(const LevelView<double> &L, const int8_t *map, double *cs, double *cn,
                              hipStream_t st)
{
    if (L.n_shared) k_shared_coef<<<blocks_for(L.n_shared), BLOCK, 0, st>>>(L, map, cs, cn);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scaled(const LevelView<T> &L, int mode, const T *u, const T *f, T *y,
                         double *partial, int *n_partial, hipStream_t st)
{
    const int gv = march_blocks(L);
    const int gs = blocks_for(L.n_shared);
    if (mode == MODE_APPLY) {
        launch_march<T, MODE_APPLY, 0>(L, u, f, y, partial, st);
        launch_shared_rows_scaled<T, MODE_APPLY>(L, u, f, y, partial, st);
    } else {
        launch_march<T, MODE_RESID, 0>(L, u, f, y, partial, st);
        launch_shared_rows_scaled<T, MODE_RESID>(L, u, f, y, partial + gv, st);
        if (n_partial) *n_partial = gv + gs;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_nodal(const LevelView<T> &L, const T *u, T *y, hipStream_t st)
{
    launch_march<T, MODE_APPLY, 1>(L, u, nullptr, y, nullptr, st);
    launch_shared_rows<T, MODE_APPLY>(L, L.sh_cn, u, nullptr, y, nullptr, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------- modification
// Row q gets sum_c delta_c (u_nb - u_self) added (MODE_APPLY) or subtracted
// from the residual (MODE_RESID, with the change of r^2 per block).
// In the fused Chebyshev mode y is the new iterate: the row's residual
// changes by -acc, so d and u_new both change by -c_r D^{-1} acc.
template <typename T, int MODE>
__global__ __launch_bounds__(BLOCK) void k_correction(CorrView<T> C, const T *__restrict__ u,
                                                      T *__restrict__ y,
                                                      double *__restrict__ partial, ChebArgs<T> cb, int nodal_mask)
{
    const int q = blockIdx.x * BLOCK + threadIdx.x;
    double dsq = 0.0;
    // rows of the primitive-mixed operator's nodal primitives are not scaled
    // rows and get no correction
    if (q < C.n_rows && !(nodal_mask && (C.c_prim[q] & nodal_mask))) {
        T acc = T(0);
        for (int c = C.c_off[q]; c < C.c_off[q + 1]; ++c)
            acc += C.c_delta[c] * (u[C.c_nb[c]] - u[C.c_self[c]]);
        const int64_t p0 = C.p_slot[C.p_off[q]];
        if (MODE == MODE_CHEB) {
            const T delta = cb.c_r * cb.invd[p0] * acc;
            const T dn = cb.d[p0] - delta, un = y[p0] - delta;
            cb.d[p0] = dn;  // d is read at the first copy only
            for (int p = C.p_off[q]; p < C.p_off[q + 1]; ++p) y[C.p_slot[p]] = un;
        } else {
            const T old = y[p0];
            const T nw = MODE == MODE_APPLY ? old + acc : old - acc;
            for (int p = C.p_off[q]; p < C.p_off[q + 1]; ++p) y[C.p_slot[p]] = nw;
            dsq = (double)nw * (double)nw - (double)old * (double)old;
        }
    }
    if (MODE == MODE_RESID) {
        dsq = block_reduce(dsq, 0);
        if (threadIdx.x == 0) partial[blockIdx.x] = dsq;
    }
}

template <typename T>
hipError_t launch_correction(const LevelView<T> &L, const CorrView<T> &C, int mode, const T *u,
                             T *y, double *partial, hipStream_t st)
{
    (void)L;
    if (!C.n_rows) return hipSuccess;
    if (mode == MODE_APPLY)
        k_correction<T, MODE_APPLY><<<blocks_for(C.n_rows), BLOCK, 0, st>>>(C, u, y, partial, ChebArgs<T>(), 0);
    else
        k_correction<T, MODE_RESID><<<blocks_for(C.n_rows), BLOCK, 0, st>>>(C, u, y, partial, ChebArgs<T>(), 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mixed(const LevelView<T> &L, const CorrView<T> &C, const T *u, T *y, int nodal_mask,
                        hipStream_t st)
{
    launch_march<T, MODE_APPLY, 0>(L, u, nullptr, y, nullptr, st);
    launch_shared_rows<T, MODE_APPLY>(L, L.sh_cs, u, nullptr, y, nullptr, st, ChebArgs<T>(), L.sh_cn, nodal_mask);
    if (C.n_rows)
        k_correction<T, MODE_APPLY><<<blocks_for(C.n_rows), BLOCK, 0, st>>>(C, u, y, nullptr, ChebArgs<T>(),
                                                                           nodal_mask);
    return hipGetLastError();
}

// the scalar nodal form (form 1) or the primitive-mixed form (form 2, nodal
// rows on the primitives in nodal_mask) in MODE_APPLY or MODE_RESID; in
// residual mode per-block sums of squares go to partial[0 .. *n_partial)
template <typename T>
hipError_t launch_scalar_form(const LevelView<T> &L, const CorrView<T> &C, int form, int mode, int nodal_mask,
                              const T *u, const T *f, T *y, double *partial, int *n_partial, hipStream_t st)
{
    const bool resid = mode == MODE_RESID;
    const int gs = blocks_for(L.n_shared);
    int gv;
    if (form == 1) {
        gv = march_grid(L.n_tet, L.vpt, L.bpt2);  // the nodal rows' one-row-per-lane grid
        if (resid) {
            launch_march<T, MODE_RESID, 1>(L, u, f, y, partial, st);
            launch_shared_rows<T, MODE_RESID>(L, L.sh_cn, u, f, y, partial + gv, st);
        } else {
            launch_march<T, MODE_APPLY, 1>(L, u, f, y, partial, st);
            launch_shared_rows<T, MODE_APPLY>(L, L.sh_cn, u, f, y, partial, st);
        }
        if (n_partial) *n_partial = gv + gs;
        return hipGetLastError();
    }
    gv = march_blocks(L);
    const int gc = blocks_for(C.n_rows);
    if (resid) {
        launch_march<T, MODE_RESID, 0>(L, u, f, y, partial, st);
        launch_shared_rows<T, MODE_RESID>(L, L.sh_cs, u, f, y, partial + gv, st, ChebArgs<T>(), L.sh_cn, nodal_mask);
        if (C.n_rows)
            k_correction<T, MODE_RESID><<<gc, BLOCK, 0, st>>>(C, u, y, partial + gv + gs, ChebArgs<T>(), nodal_mask);
    } else {
        launch_march<T, MODE_APPLY, 0>(L, u, f, y, partial, st);
        launch_shared_rows<T, MODE_APPLY>(L, L.sh_cs, u, f, y, partial, st, ChebArgs<T>(), L.sh_cn, nodal_mask);
        if (C.n_rows)
            k_correction<T, MODE_APPLY><<<gc, BLOCK, 0, st>>>(C, u, y, partial, ChebArgs<T>(), nodal_mask);
    }
    if (n_partial) *n_partial = gv + gs + (C.n_rows ? gc : 0);
    return hipGetLastError();
}


template <typename T>
hipError_t launch_cheb_sweep(const LevelView<T> &L, const CorrView<T> &C, const T *u, const T *f, T *u_new,
                             const ChebArgs<T> &cb, hipStream_t st)
{
    launch_march<T, MODE_CHEB, 0>(L, u, f, u_new, nullptr, st, cb);
    launch_shared_rows_scaled<T, MODE_CHEB>(L, u, f, u_new, nullptr, st, cb);
    if (C.n_rows)
        k_correction<T, MODE_CHEB><<<blocks_for(C.n_rows), BLOCK, 0, st>>>(C, u, u_new, nullptr, cb, 0);
    return hipGetLastError();
}

// the same fused sweep for the primitive-mixed form: nodal coefficients on
// the shared rows of the primitives in nodal_mask, whose modification rows
// are skipped.  (A fused sweep of the nodal form needs 244 registers per lane
// and ran slower than its residual plus update passes.)
template <typename T>
hipError_t launch_cheb_sweep_mixed(const LevelView<T> &L, const CorrView<T> &C, int nodal_mask, const T *u,
                                   const T *f, T *u_new, const ChebArgs<T> &cb, hipStream_t st)
{
    launch_march<T, MODE_CHEB, 0>(L, u, f, u_new, nullptr, st, cb);
    launch_shared_rows<T, MODE_CHEB>(L, L.sh_cs, u, f, u_new, nullptr, st, cb, L.sh_cn, nodal_mask);
    if (C.n_rows)
        k_correction<T, MODE_CHEB><<<blocks_for(C.n_rows), BLOCK, 0, st>>>(C, u, u_new, nullptr, cb, nodal_mask);
    return hipGetLastError();
}

// ---------------------------------------------------------------- diagonal
// D_i = -sum_d w_d (k_i + k_{i+d}); per row the Gershgorin ratio
// 1 + sum over tets and directions of |entry| / D_i (entries to Dirichlet
// nodes excluded); block maxima go to `partial`.
__device__ __forceinline__ bool is_dirichlet(const uint16_t *dmask, int tet, int n, int i, int j, int k)
{
    return (dmask[tet] >> zero_pattern(n, i, j, k)) & 1;
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_diag_volume(LevelView<T> L, T *__restrict__ dout,
                                                        double *__restrict__ asum_out,
                                                        double *__restrict__ partial)
{
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    double g = 0.0;
    if (lb < L.n_tet * L.bpt) {
        const int tet = lb / L.bpt;
        const int s = (lb - tet * L.bpt) * BLOCK + threadIdx.x;
        if (s < L.S) {
            const int64_t base = (int64_t)tet * L.Spad;
            int i, j, k;
            decode_slot(L.n, s, i, j, k);
            if (i == 0 || j == 0 || k == 0 || i + j + k == L.n) {
                if (is_dirichlet(L.dmask, tet, L.n, i, j, k)) dout[base + s] = T(0);
            } else {
                const T *w = L.sten + (int64_t)tet * TET_STENCIL;
                int nb[NDIR];
                neighbour_slots(s, i + j, L.n - k, nb);
                const double k0 = (double)L.kap[base + s];
                double dsum = 0.0, asum = 0.0;
                for (int d = 0; d < NDIR; ++d) {
                    const double e = (double)w[d] * (k0 + (double)L.kap[base + nb[d]]);
                    dsum -= e;
                    if (!is_dirichlet(L.dmask, tet, L.n, i + DIR[d][0], j + DIR[d][1], k + DIR[d][2]))
                        asum += fabs(e);
                }
                dout[base + s] = (T)dsum;
                if (asum_out) asum_out[base + s] = asum;
                g = 1.0 + asum / dsum;
            }
        }
    }
    g = block_reduce(g, 1);
    if (threadIdx.x == 0) partial[blockIdx.x] = g;
}

// shared rows: D and the Gershgorin absolute row sum (sum over copies and
// directions) into every copy, and (asum, D) per shared node into gabs
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_diag_shared(LevelView<T> L, T *__restrict__ dout,
                                                        double *__restrict__ asum_out,
                                                        double *__restrict__ gabs)
{
    const int q = blockIdx.x * BLOCK + threadIdx.x;
    if (q >= L.n_shared) return;
    double dsum = 0.0, asum = 0.0;
    for (int c = L.sh_off[q]; c < L.sh_off[q + 1]; ++c) {
        int tet, kind, i, j, k;
        unpack_copy(L.sh_copy[c], tet, kind, i, j, k);
        const int64_t base = (int64_t)tet * L.Spad;
        const int s = slot32(L.n, i, j, k);
        int nb[NDIR];
        neighbour_slots(s, i + j, L.n - k, nb);
        const T *w = L.sten + (int64_t)tet * TET_STENCIL + kind * KIND_STRIDE;
        const double k0 = (double)L.kap[base + s];
        for (int d = 0; d < NDIR; ++d) {
            if (w[d] == T(0)) continue;
            const double e = (double)w[d] * (k0 + (double)L.kap[base + nb[d]]);
            dsum -= e;
            if (!is_dirichlet(L.dmask, tet, L.n, i + DIR[d][0], j + DIR[d][1], k + DIR[d][2]))
                asum += fabs(e);
        }
    }
    for (int c = L.sh_off[q]; c < L.sh_off[q + 1]; ++c) {
        int tet, kind, i, j, k;
        unpack_copy(L.sh_copy[c], tet, kind, i, j, k);
        const int64_t sl = (int64_t)tet * L.Spad + slot32(L.n, i, j, k);
        dout[sl] = (T)dsum;
        if (asum_out) asum_out[sl] = asum;
    }
    gabs[2 * q] = asum;
    gabs[2 * q + 1] = dsum;
}

template <typename T>
hipError_t launch_diag(const LevelView<T> &L, T *d, double *asum, double *partial, double *gabs,
                       int *n_partial, hipStream_t st)
{
    const int gv = volume_grid(L.n_tet, L.bpt);
    k_diag_volume<T><<<gv, BLOCK, 0, st>>>(L, d, asum, partial);
    if (L.n_shared) k_diag_shared<T><<<blocks_for(L.n_shared), BLOCK, 0, st>>>(L, d, asum, gabs);
    *n_partial = gv;
    return hipGetLastError();
}

// ---------------------------------------------------------------- reductions
__global__ __launch_bounds__(BLOCK) void k_reduce(const double *__restrict__ p, int n, int op_max,
                                                  double *__restrict__ out)
{
    double v = op_max ? -1e300 : 0.0;
    for (int q = threadIdx.x; q < n; q += BLOCK) v = op_max ? fmax(v, p[q]) : v + p[q];
    v = block_reduce(v, op_max);
    if (threadIdx.x == 0) *out = v;
}

hipError_t launch_reduce(const double *partial, int n, int op_max, double *out, hipStream_t st)
{
    k_reduce<<<1, BLOCK, 0, st>>>(partial, n, op_max, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- vector updates
template <typename T>
__global__ void k_invert(T *d, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n) d[q] = d[q] != T(0) ? T(1) / d[q] : T(0);
}
template <typename T>
hipError_t launch_invert_diag(T *d, int64_t n, hipStream_t st)
{
    k_invert<T><<<blocks_for(n), BLOCK, 0, st>>>(d, n);
    return hipGetLastError();
}

template <typename T>
__global__ void k_jacobi(T *__restrict__ u, const T *__restrict__ r, const T *__restrict__ invd,
                         T omega, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n) u[q] += omega * invd[q] * r[q];
}
template <typename T>
hipError_t launch_jacobi_update(T *u, const T *r, const T *invd, T omega, int64_t n, hipStream_t st)
{
    k_jacobi<T><<<blocks_for(n), BLOCK, 0, st>>>(u, r, invd, omega, n);
    return hipGetLastError();
}

// Chebyshev step: d <- c_old d + c_r D^{-1} r ; u <- u + d
template <typename T>
__global__ void k_cheb(T *__restrict__ u, T *__restrict__ dv, const T *__restrict__ r,
                       const T *__restrict__ invd, T c_old, T c_r, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n) {
        const T d = (c_old != T(0) ? c_old * dv[q] : T(0)) + c_r * invd[q] * r[q];
        dv[q] = d;
        u[q] += d;
    }
}
template <typename T>
hipError_t launch_cheb_update(T *u, T *dvec, const T *r, const T *invd, T c_old, T c_r,
                              int64_t n, hipStream_t st)
{
    k_cheb<T><<<blocks_for(n), BLOCK, 0, st>>>(u, dvec, r, invd, c_old, c_r, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------- grid transfer
// restriction = transpose of P1 interpolation: r_c(x) = r_f(2x) + 1/2 sum_d r_f(2x+d)
// grids over (in-plane chunk, plane k, tet): a thread finds its lattice point
// from its in-plane offset alone (threads past the plane's end return)
__device__ __forceinline__ bool plane_point(int n, int &i, int &j, int &k, int &s)
{
    k = blockIdx.y;
    const int t = blockIdx.x * BLOCK + threadIdx.x;
    if (t >= tr32(n - k)) return false;
    int d = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((d + 1) * (d + 2) / 2 <= t) ++d;
    while (d > 0 && d * (d + 1) / 2 > t) --d;
    i = t - d * (d + 1) / 2;
    j = d - i;
    s = tc32(n) - tc32(n - k) + t;
    return true;
}
static inline dim3 plane_grid(int n, int n_tet) { return dim3((unsigned)((tri_count(n) + BLOCK - 1) / BLOCK), (unsigned)(n + 1), (unsigned)n_tet); }

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_restrict_volume(LevelView<T> Lc, LevelView<T> Lf,
                                                            const T *__restrict__ rf,
                                                            T *__restrict__ rc)
{
    int i, j, k, s;
    if (!plane_point(Lc.n, i, j, k, s)) return;
    const int tet = blockIdx.z;
    const int64_t bc = (int64_t)tet * Lc.Spad;
    if (i == 0 || j == 0 || k == 0 || i + j + k == Lc.n) {
        if (is_dirichlet(Lc.dmask, tet, Lc.n, i, j, k)) rc[bc + s] = T(0);
        return;
    }
    const T *__restrict__ fb = rf + (int64_t)tet * Lf.Spad;
    const int sf = slot32(Lf.n, 2 * i, 2 * j, 2 * k);
    int nb[NDIR];
    neighbour_slots(sf, 2 * (i + j), Lf.n - 2 * k, nb);
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < NDIR; ++d) acc += fb[nb[d]];
    rc[bc + s] = fb[sf] + T(0.5) * acc;
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_restrict_shared(LevelView<T> Lc, LevelView<T> Lf,
                                                            const T *__restrict__ rf,
                                                            T *__restrict__ rc)
{
    const int q = blockIdx.x * BLOCK + threadIdx.x;
    if (q >= Lc.n_shared) return;
    T acc = T(0);
    // a direction with weight 0 (outside the copy's tet) gathers the centre
    // instead and adds an exact zero, so every gather of a copy is issued at
    // once (no branch per direction)
#pragma unroll 2
    for (int c = Lc.sh_off[q]; c < Lc.sh_off[q + 1]; ++c) {
        int tet, kind, i, j, k;
        unpack_copy(Lc.sh_copy[c], tet, kind, i, j, k);
        const T *fb = rf + (int64_t)tet * Lf.Spad;
        const T *w = Lc.rstw + (int64_t)tet * TET_STENCIL + kind * KIND_STRIDE;
        const int sf = slot32(Lf.n, 2 * i, 2 * j, 2 * k);
        int nb[NDIR];
        neighbour_slots(sf, 2 * (i + j), Lf.n - 2 * k, nb);
        T wv[NDIR + 1], fv[NDIR + 1];
#pragma unroll
        for (int d = 0; d <= NDIR; ++d) wv[d] = w[d];
#pragma unroll
        for (int d = 0; d < NDIR; ++d) fv[d] = fb[wv[d] != T(0) ? nb[d] : sf];
        fv[NDIR] = fb[sf];
        acc += wv[NDIR] * fv[NDIR];
#pragma unroll
        for (int d = 0; d < NDIR; ++d) acc += wv[d] * fv[d];
    }
    for (int c = Lc.sh_off[q]; c < Lc.sh_off[q + 1]; ++c) {
        int tet, kind, i, j, k;
        unpack_copy(Lc.sh_copy[c], tet, kind, i, j, k);
        rc[(int64_t)tet * Lc.Spad + slot32(Lc.n, i, j, k)] = acc;
    }
}

template <typename T>
hipError_t launch_restrict(const LevelView<T> &Lc, const LevelView<T> &Lf, const T *rf, T *rc,
                           hipStream_t st)
{
    k_restrict_volume<T><<<plane_grid(Lc.n, Lc.n_tet), BLOCK, 0, st>>>(Lc, Lf, rf, rc);
    if (Lc.n_shared) k_restrict_shared<T><<<blocks_for(Lc.n_shared), BLOCK, 0, st>>>(Lc, Lf, rf, rc);
    return hipGetLastError();
}

// P1 interpolation and add: a fine node with all-even lattice coordinates is a
// coarse node; any other fine node is the midpoint of the coarse edge whose
// direction has the parity pattern of (i, j, k): (i odd) -> (1,0,0),
// (j) -> (0,1,0), (i,j) -> (1,-1,0), (k) -> (0,0,1), (i,k) -> (1,0,-1),
// (j,k) -> (0,1,-1), (i,j,k) -> (1,-1,1).
// Column marching: a lane owns one in-plane
// position t = (s, i) of the fine lattice and walks a chunk of planes; its
// coarse in-plane offsets are fixed per plane parity (even planes: both
// edge ends in coarse plane k/2; odd planes: one end in plane (k-1)/2, the
// other in (k+1)/2), so a plane costs the fine read-modify-write and two
// coarse reads with no per-point index arithmetic.
constexpr int PKC = 16;  // fine planes per wave

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_prolong_march(LevelView<T> Lc, LevelView<T> Lf,
                                                          const T *__restrict__ uc, T *__restrict__ uf,
                                                          int n_seg)
{
    const int tet = blockIdx.y;
    const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6));
    const int ch = w / n_seg, seg = w - ch * n_seg;
    const int n = Lf.n, nc = Lc.n;
    const int k0 = ch * PKC;
    const int t0 = seg * 64;
    auto diag = [](int t) {
        int d = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while ((d + 1) * (d + 2) / 2 <= t) ++d;
        while (d > 0 && d * (d + 1) / 2 > t) --d;
        return d;
    };
    // whole wave: chunk past the top or past every column of the segment
    if (k0 > n || k0 > n - diag(t0)) return;
    const int k1 = min(n, k0 + PKC - 1);
    const int t = t0 + (int)(threadIdx.x & 63);
    const int s = diag(t), i = t - s * (s + 1) / 2, j = s - i;
    const int kmax = t < tr32(n) ? n - s : -1;  // last plane holding this column
    const int pi = i & 1, pj = j & 1;
    auto off = [](int a, int b) { return (a + b) * (a + b + 1) / 2 + a; };
    // even planes: direction (pi, pj ? (pi ? -1 : 1) : 0, 0)
    const int dje = pj ? (pi ? -1 : 1) : 0;
    const int ea = off((i - pi) >> 1, (j - dje) >> 1), eb = off((i + pi) >> 1, (j + dje) >> 1);
    // odd planes: k component +1 for (0,0) and (1,1) parities, -1 otherwise;
    // lo is the end in the lower coarse plane
    const int dko = (pi == pj) ? 1 : -1;
    const int lo_i = dko == 1 ? (i - pi) >> 1 : (i + pi) >> 1, lo_j = dko == 1 ? (j - dje) >> 1 : (j + dje) >> 1;
    const int hi_i = dko == 1 ? (i + pi) >> 1 : (i - pi) >> 1, hi_j = dko == 1 ? (j + dje) >> 1 : (j - dje) >> 1;
    const int olo = off(lo_i, lo_j), ohi = off(hi_i, hi_j);
    constexpr int B = (int)sizeof(T);
    const __amdgpu_buffer_rsrc_t rc = tet_rsrc(uc + (int64_t)tet * Lc.Spad, (int64_t)Lc.S * B);
    const __amdgpu_buffer_rsrc_t rf = tet_rsrc(uf + (int64_t)tet * Lf.Spad, (int64_t)Lf.S * B);
    const int Sf = tc32(n), Sc = tc32(nc);
    constexpr int DROP = 0x7ffffff0;
#pragma unroll 4
    for (int k = k0; k <= k1; ++k) {
        const int fs = Sf - tc32(n - k) + t;
        int ca, cb;
        if (k & 1) {
            ca = Sc - tc32(nc - ((k - 1) >> 1)) + olo;
            cb = Sc - tc32(nc - ((k + 1) >> 1)) + ohi;
        } else {
            const int P = Sc - tc32(nc - (k >> 1));
            ca = P + ea;
            cb = P + eb;
        }
        const T a = bload<T>(rc, ca), b = bload<T>(rc, cb);
        const T old = bload<T>(rf, fs);
        bstore(old + T(0.5) * (a + b), rf, k <= kmax ? fs * B : DROP);
    }
}

template <typename T>
hipError_t launch_prolong_add(const LevelView<T> &Lc, const LevelView<T> &Lf, const T *uc, T *uf,
                              hipStream_t st)
{
    const int n = Lf.n;
    const int n_seg = (int)((tri_count(n) + 63) / 64);
    const int waves = n_seg * ((n + PKC) / PKC);
    k_prolong_march<T><<<dim3((unsigned)((waves + BLOCK / 64 - 1) / (BLOCK / 64)), (unsigned)Lf.n_tet), BLOCK, 0,
                         st>>>(Lc, Lf, uc, uf, n_seg);
    return hipGetLastError();
}

// ---------------------------------------------------------------- stored stencils
// Interior rows by column marching (a lane owns one in-plane offset t and
// walks a chunk of planes; neighbour slots from neighbour_slots with the
// plane's size).  Filling stores c_d = w_d (k_0 + k_d) for the 14 directions
// (the scaled row's coefficients, eq. (discrete) with the half reference
// entries) and the centre -sum_d c_d; the apply is the plain 15-term product
// of the stored row with u.
constexpr int SKC = 16;  // planes per wave

__device__ __forceinline__ bool stored_lane(int n, int n_seg, int &t, int &sd, int &k0, int &k1, int &tet)
{
    tet = blockIdx.y;
    const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6));
    const int ch = w / n_seg, seg = w - ch * n_seg;
    k0 = ch * SKC + 1;
    if (k0 > n - 3) return false;
    k1 = min(n - 3, k0 + SKC - 1);
    t = seg * 64 + (int)(threadIdx.x & 63);
    int d = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((d + 1) * (d + 2) / 2 <= t) ++d;
    while (d > 0 && d * (d + 1) / 2 > t) --d;
    sd = d;
    return true;
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_store_stencil(LevelView<double> L, T *__restrict__ st, int n_seg)
{
    int t, sd, k0, k1, tet;
    const int n = L.n;
    if (!stored_lane(n, n_seg, t, sd, k0, k1, tet)) return;
    const int i = t - sd * (sd + 1) / 2, j = sd - i;
    if (i < 1 || j < 1) return;
    const int64_t base = (int64_t)tet * L.Spad;
    const double *__restrict__ kb = L.kap + base;
    const double *w = L.sten + (int64_t)tet * TET_STENCIL;
    T *__restrict__ sb = st + (int64_t)tet * 15 * L.Spad;
    const int Sn = tc32(n);
    for (int k = k0; k <= min(k1, n - 1 - sd); ++k) {
        const int s = Sn - tc32(n - k) + t;
        int nb[NDIR];
        neighbour_slots(s, sd, n - k, nb);
        const double k0v = kb[s];
        double diag = 0.0;
        for (int d = 0; d < NDIR; ++d) {
            const double c = w[d] * (k0v + kb[nb[d]]);
            sb[(int64_t)d * L.Spad + s] = (T)c;
            diag -= c;
        }
        sb[(int64_t)NDIR * L.Spad + s] = (T)diag;
    }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_stored_apply(LevelView<T> L, const T *__restrict__ st,
                                                         const T *__restrict__ u, T *__restrict__ y, int n_seg)
{
    int t, sd, k0, k1, tet;
    const int n = L.n;
    if (!stored_lane(n, n_seg, t, sd, k0, k1, tet)) return;
    const int i = t - sd * (sd + 1) / 2, j = sd - i;
    if (i < 1 || j < 1) return;
    const int64_t base = (int64_t)tet * L.Spad;
    const T *__restrict__ ub = u + base;
    const T *__restrict__ sb = st + (int64_t)tet * 15 * L.Spad;
    const int Sn = tc32(n);
#pragma unroll 2
    for (int k = k0; k <= min(k1, n - 1 - sd); ++k) {
        const int s = Sn - tc32(n - k) + t;
        int nb[NDIR];
        neighbour_slots(s, sd, n - k, nb);
        T acc = sb[(int64_t)NDIR * L.Spad + s] * ub[s];
#pragma unroll
        for (int d = 0; d < NDIR; ++d) acc += sb[(int64_t)d * L.Spad + s] * ub[nb[d]];
        y[base + s] = acc;
    }
}

// ---------------------------------------------------------------- tensor coefficient
// Row of node 0: sum_m sum_d w^m_d (k_m,0 + k_m,d) (u_d - u_0) with the
// half reference entries w^m of component m (Sec. 2.1 eq. (integral), each
// a_m scaled as the scalar form).  On interior rows w^m_d = w^m_{d+7}, so the
// coefficient of direction d is K_p(node 0) + K_p(node d) with the pair field
// K_p = sum_m w^m_p k_m (p = d mod 7), formed once per coefficient: seven
// fields and 28 neighbour gathers per row instead of six fields and 90.
// Inter-tet rows take merged coefficients (k_tensor_shared_coef) like the
// scalar operator's.
__global__ void k_tensor_pairs(LevelView<double> L, double *__restrict__ kp)
{
    const int64_t ns = (int64_t)L.n_tet * L.Spad;
    const int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (e >= ns) return;
    const int tet = (int)(e / L.Spad);
    double km[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) km[m] = L.kt[m * ns + e];
#pragma unroll
    for (int p = 0; p < NDIR / 2; ++p) {
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) acc += L.tsten[((int64_t)tet * 6 + m) * TET_STENCIL + p] * km[m];
        kp[p * ns + e] = acc;
    }
}

// MODE_APPLY: y = A u; MODE_RESID: y = f - A u and the block's sum of
// squares in partial (one entry per block of the 2D grid)
template <typename T, int MODE>
__global__ __launch_bounds__(BLOCK) void k_tensor_interior(LevelView<T> L, const T *__restrict__ u,
                                                            const T *__restrict__ f, T *__restrict__ y,
                                                            double *__restrict__ partial, int n_seg)
{
    int t = 0, sd = 0, k0 = 0, k1 = -1, tet;
    const int n = L.n;
    double sq = 0.0;
    if (stored_lane(n, n_seg, t, sd, k0, k1, tet)) {
        const int i = t - sd * (sd + 1) / 2, j = sd - i;
        if (i >= 1 && j >= 1) {
            const int64_t base = (int64_t)tet * L.Spad, ns = (int64_t)L.n_tet * L.Spad;
            const T *__restrict__ ub = u + base;
            const T *__restrict__ kb = L.kp + base;
            const int Sn = tc32(n);
#pragma unroll 2
            for (int k = k0; k <= min(k1, n - 1 - sd); ++k) {
                const int s = Sn - tc32(n - k) + t;
                int nb[NDIR];
                neighbour_slots(s, sd, n - k, nb);
                const T u0 = ub[s];
                T acc = T(0);
#pragma unroll
                for (int p = 0; p < NDIR / 2; ++p) {
                    const T *__restrict__ kq = kb + p * ns;
                    const int a = nb[p], b = nb[p + NDIR / 2];
                    const T c0 = kq[s];
                    acc += (c0 + kq[a]) * (ub[a] - u0) + (c0 + kq[b]) * (ub[b] - u0);
                }
                if (MODE == MODE_RESID) {
                    acc = f[base + s] - acc;
                    sq += (double)acc * (double)acc;
                }
                y[base + s] = acc;
            }
        }
    }
    if (MODE == MODE_RESID) {
        sq = block_reduce(sq, 0);
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = sq;
    }
}

// Nodal-integration tensor operator: per component the row of eq.
// (standardfe) with that component's element matrices and field, summed over
// the six components.  Interior rows gather u and each k_m over the 15-point
// neighbourhood (all 24 incident elements lie in the tet); inter-tet rows take
// merged coefficients (k_tensor_shared_coef).  Modes as k_tensor_interior.
template <typename T, int MODE>
__global__ __launch_bounds__(BLOCK) void k_tensor_nodal_interior(LevelView<T> L, const T *__restrict__ u,
                                                                  const T *__restrict__ f, T *__restrict__ y,
                                                                  double *__restrict__ partial, int n_seg)
{
    __shared__ T es[6 * TET_EMAT];
    for (int q = threadIdx.x; q < 6 * TET_EMAT; q += BLOCK)
        es[q] = L.temat[(int64_t)blockIdx.y * 6 * TET_EMAT + q];
    __syncthreads();
    int t = 0, sd = 0, k0 = 0, k1 = -1, tet;
    const int n = L.n;
    double sq = 0.0;
    if (stored_lane(n, n_seg, t, sd, k0, k1, tet)) {
        const int i = t - sd * (sd + 1) / 2, j = sd - i;
        if (i >= 1 && j >= 1) {
            const int64_t base = (int64_t)tet * L.Spad, ns = (int64_t)L.n_tet * L.Spad;
            const T *__restrict__ ub = u + base;
            const int Sn = tc32(n);
#pragma unroll 1
            for (int k = k0; k <= min(k1, n - 1 - sd); ++k) {
                const int s = Sn - tc32(n - k) + t;
                int nb[NDIR];
                neighbour_slots(s, sd, n - k, nb);
                T uu[NDIR + 1];
#pragma unroll
                for (int d = 0; d < NDIR; ++d) uu[d] = ub[nb[d]];
                uu[NDIR] = ub[s];
                T acc = T(0);
#pragma unroll 1
                for (int m = 0; m < 6; ++m) {
                    const T *__restrict__ km = L.kt + m * ns + base;
                    T kk[NDIR + 1];
#pragma unroll
                    for (int d = 0; d < NDIR; ++d) kk[d] = km[nb[d]];
                    kk[NDIR] = km[s];
                    acc += row_value<T, 1>(uu, kk, es + m * TET_EMAT);
                }
                if (MODE == MODE_RESID) {
                    acc = f[base + s] - acc;
                    sq += (double)acc * (double)acc;
                }
                y[base + s] = acc;
            }
        }
    }
    if (MODE == MODE_RESID) {
        sq = block_reduce(sq, 0);
        if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = sq;
    }
}

// Diagonal of a form on interior rows (FP64, at set-up): FORM 0 the scaled
// tensor form, 1 the nodal tensor form, 2 the scalar nodal form.  With the
// row written as sum_d c_d (u_d - u_0), a_00 = -sum_d c_d and a_0d = c_d.
// Stores a_00 in diag and the block's largest Gershgorin bound
// 1 + sum_d |c_d| / a_00 of D^{-1} A in partial.
template <int FORM>
__global__ __launch_bounds__(BLOCK) void k_form_diag(LevelView<double> L, double *__restrict__ diag,
                                                     double *__restrict__ partial, int n_seg)
{
    int t = 0, sd = 0, k0 = 0, k1 = -1, tet;
    const int n = L.n;
    double g = 0.0;
    if (stored_lane(n, n_seg, t, sd, k0, k1, tet)) {
        const int i = t - sd * (sd + 1) / 2, j = sd - i;
        if (i >= 1 && j >= 1) {
            const int64_t base = (int64_t)tet * L.Spad, ns = (int64_t)L.n_tet * L.Spad;
            const int Sn = tc32(n);
            for (int k = k0; k <= min(k1, n - 1 - sd); ++k) {
                const int s = Sn - tc32(n - k) + t;
                int nb[NDIR];
                neighbour_slots(s, sd, n - k, nb);
                double cd[NDIR];
                for (int d = 0; d < NDIR; ++d) cd[d] = 0.0;
                if (FORM == 0) {
                    for (int d = 0; d < NDIR; ++d) {
                        const double *kq = L.kp + (d % (NDIR / 2)) * ns + base;
                        cd[d] = kq[s] + kq[nb[d]];
                    }
                } else {
                    // FORM 1: six components; FORM 2: the scalar k and element matrices
                    for (int m = 0; m < (FORM == 1 ? 6 : 1); ++m) {
                        const double *km = (FORM == 1 ? L.kt + m * ns : L.kap) + base;
                        double kk[NDIR + 1];
                        for (int d = 0; d < NDIR; ++d) kk[d] = km[nb[d]];
                        kk[NDIR] = km[s];
                        const double *w = FORM == 1 ? L.temat + ((int64_t)tet * 6 + m) * TET_EMAT
                                                    : L.emat + (int64_t)tet * TET_EMAT;
                        for (int ty = 0; ty < NTYPE; ++ty)
                            for (int a = 0; a < 4; ++a) {
                                double ks = 0.0;
                                for (int v = 0; v < 4; ++v) ks += kk[ELEM_DIR.v[ty][a][v]];
                                for (int v = 0; v < 4; ++v) {
                                    const int d = ELEM_DIR.v[ty][a][v];
                                    if (d != NDIR) cd[d] += ks * w[ty * 16 + a * 4 + v];
                                }
                            }
                    }
                }
                double dg = 0.0, ab = 0.0;
                for (int d = 0; d < NDIR; ++d) {
                    dg -= cd[d];
                    ab += fabs(cd[d]);
                }
                diag[base + s] = dg;
                g = fmax(g, 1.0 + ab / dg);
            }
        }
    }
    g = block_reduce(g, 1);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = g;
}

// the same for shared rows from merged coefficients of `width` entries,
// written to every copy; with a nonzero mask only the rows of nodes on those
// macro primitives
__global__ __launch_bounds__(BLOCK) void k_shared_diag(LevelView<double> L, const double *__restrict__ coef,
                                                       int width, int mask, double *__restrict__ diag,
                                                       double *__restrict__ partial)
{
    const int q = blockIdx.x * BLOCK + threadIdx.x;
    double g = 0.0;
    if (q < L.n_shared && (!mask || (L.sh_prim[q] & mask))) {
        double dg = 0.0, ab = 0.0;
        for (int e = 0; e < width; ++e) {
            const double c = coef[(int64_t)e * L.n_shared + q];
            dg -= c;
            ab += fabs(c);
        }
        for (int c = L.sh_off[q]; c < L.sh_off[q + 1]; ++c) diag[L.sh_cslot[c]] = dg;
        g = 1.0 + ab / dg;
    }
    g = block_reduce(g, 1);
    if (threadIdx.x == 0) partial[blockIdx.x] = g;
}

// merged coefficients of the tensor operator's shared rows (FP64, once per
// tensor coefficient), on the tensor operator's sparsity pattern:
// scaled  c_e = sum over copies, components m and directions d onto e of
//         w^m_d (k_m,q + k_m,e) with the copy's tet-restricted stencils;
// nodal   c_e = sum over copies, elements t holding the node and m of
//         (sum of k_m at t's vertices) (A^m_t / 4)[node, e]
__global__ __launch_bounds__(BLOCK) void k_tensor_shared_coef(LevelView<double> L, const int8_t *__restrict__ map,
                                                              double *__restrict__ cs, double *__restrict__ cn)
{
    const int q = blockIdx.x * BLOCK + threadIdx.x;
    const int ns = L.n_shared;
    if (q >= ns) return;
    const int64_t nsl = (int64_t)L.n_tet * L.Spad;
    for (int e = 0; e < L.sh_w; ++e) {
        cs[(int64_t)e * ns + q] = 0.0;
        cn[(int64_t)e * ns + q] = 0.0;
    }
    for (int c = L.sh_off[q]; c < L.sh_off[q + 1]; ++c) {
        int tet, kind, i, j, k;
        unpack_copy(L.sh_copy[c], tet, kind, i, j, k);
        const int64_t base = (int64_t)tet * L.Spad;
        const int s = slot32(L.n, i, j, k);
        const int8_t *mp = map + (int64_t)c * 16;
        int nb[NDIR];
        neighbour_slots(s, i + j, L.n - k, nb);
        for (int m = 0; m < 6; ++m) {
            const double *km = L.kt + m * nsl + base;
            const double *w = L.tsten + ((int64_t)tet * 6 + m) * TET_STENCIL + kind * KIND_STRIDE;
            for (int d = 0; d < NDIR; ++d) {
                const int e = mp[d];
                if (e >= 0 && w[d] != 0.0) cs[(int64_t)e * ns + q] += w[d] * (km[s] + km[nb[d]]);
            }
        }
        for (int t = 0; t < NTYPE; ++t)
            for (int a = 0; a < 4; ++a) {
                // element of shape t whose vertex a is this node
                int sl[4];
                bool ok = true;
                for (int v = 0; v < 4; ++v) {
                    const int d = ELEM_DIR.v[t][a][v];
                    if (d == NDIR) { sl[v] = s; continue; }
                    ok = ok && in_lattice(L.n, i + DIR[d][0], j + DIR[d][1], k + DIR[d][2]);
                    sl[v] = nb[d];
                }
                if (!ok) continue;
                for (int m = 0; m < 6; ++m) {
                    const double *km = L.kt + m * nsl + base;
                    const double ks = (km[sl[0]] + km[sl[1]]) + (km[sl[2]] + km[sl[3]]);
                    const double *E = L.temat + ((int64_t)tet * 6 + m) * TET_EMAT + t * 16 + a * 4;
                    for (int v = 0; v < 4; ++v) {
                        if (v == a) continue;
                        const int e = mp[ELEM_DIR.v[t][a][v]];
                        if (e >= 0) cn[(int64_t)e * ns + q] += ks * E[v];
                    }
                }
            }
    }
}

hipError_t launch_tensor_shared_coef(const LevelView<double> &L, const int8_t *map, double *cs, double *cn,
                                     hipStream_t st)
{
    LevelView<double> Lt = L;
    Lt.sh_w = L.sh_wt;
    Lt.sh_nb = L.sh_nbt;
    Lt.sh_nb32 = nullptr;
    if (L.n_shared) k_tensor_shared_coef<<<blocks_for(L.n_shared), BLOCK, 0, st>>>(Lt, map, cs, cn);
    return hipGetLastError();
}

// Dirichlet slots of y to 0 (the marches do this in their boundary blocks)
template <typename T>
__global__ void k_dirichlet_zero(LevelView<T> L, T *__restrict__ y)
{
    const int64_t e = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (e >= (int64_t)L.n_tet * L.n_bnd) return;
    const int tet = (int)(e / L.n_bnd);
    const uint32_t v = L.bnd[e - (int64_t)tet * L.n_bnd];
    if ((L.dmask[tet] >> (v & 15u)) & 1) y[(int64_t)tet * L.Spad + (v >> 4)] = T(0);
}

static inline dim3 stored_grid(int n, int n_tet, int &n_seg)
{
    n_seg = (int)((tri_count(n) + 63) / 64);
    const int chunks = n > 3 ? (n - 3 + SKC - 1) / SKC : 0;
    return dim3((unsigned)((n_seg * chunks + BLOCK / 64 - 1) / (BLOCK / 64)), (unsigned)n_tet);
}

template <typename T>
hipError_t launch_store_stencils(const LevelView<double> &L, T *st, hipStream_t strm)
{
    int n_seg = 0;
    const dim3 g = stored_grid(L.n, L.n_tet, n_seg);
    if (g.x) k_store_stencil<T><<<g, BLOCK, 0, strm>>>(L, st, n_seg);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stored(const LevelView<T> &L, const CorrView<T> &C, const T *st, const T *u, T *y,
                         hipStream_t strm)
{
    int n_seg = 0;
    const dim3 g = stored_grid(L.n, L.n_tet, n_seg);
    if (g.x) k_stored_apply<T><<<g, BLOCK, 0, strm>>>(L, st, u, y, n_seg);
    launch_shared_rows_scaled<T, MODE_APPLY>(L, u, nullptr, y, nullptr, strm);
    const int64_t nb = (int64_t)L.n_tet * L.n_bnd;
    if (nb) k_dirichlet_zero<T><<<blocks_for(nb), BLOCK, 0, strm>>>(L, y);
    if (C.n_rows)
        k_correction<T, MODE_APPLY><<<blocks_for(C.n_rows), BLOCK, 0, strm>>>(C, u, y, nullptr, ChebArgs<T>(), 0);
    return hipGetLastError();
}
hipError_t launch_tensor_pairs(const LevelView<double> &L, double *kp, hipStream_t st)
{
    const int64_t ns = (int64_t)L.n_tet * L.Spad;
    if (ns) k_tensor_pairs<<<blocks_for(ns), BLOCK, 0, st>>>(L, kp);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_tensor(const LevelView<T> &L, int form, int mode, const T *u, const T *f, T *y, double *partial,
                         int *n_partial, hipStream_t st)
{
    int n_seg = 0;
    const dim3 g = stored_grid(L.n, L.n_tet, n_seg);
    const int gi = (int)(g.x * g.y);
    const bool resid = mode == MODE_RESID;
    if (g.x) {
        if (form == 0 && !resid) k_tensor_interior<T, MODE_APPLY><<<g, BLOCK, 0, st>>>(L, u, f, y, partial, n_seg);
        if (form == 0 && resid) k_tensor_interior<T, MODE_RESID><<<g, BLOCK, 0, st>>>(L, u, f, y, partial, n_seg);
        if (form != 0 && !resid)
            k_tensor_nodal_interior<T, MODE_APPLY><<<g, BLOCK, 0, st>>>(L, u, f, y, partial, n_seg);
        if (form != 0 && resid)
            k_tensor_nodal_interior<T, MODE_RESID><<<g, BLOCK, 0, st>>>(L, u, f, y, partial, n_seg);
    }
    LevelView<T> Lt = L;  // the tensor pattern
    Lt.sh_w = L.sh_wt;
    Lt.sh_nb = L.sh_nbt;
    Lt.sh_nb32 = nullptr;
    const T *coef = form == 0 ? L.sh_ct : L.sh_ctn;
    if (resid) launch_shared_rows<T, MODE_RESID>(Lt, coef, u, f, y, partial + gi, st);
    else launch_shared_rows<T, MODE_APPLY>(Lt, coef, u, f, y, nullptr, st);
    const int64_t nb = (int64_t)L.n_tet * L.n_bnd;
    if (nb) k_dirichlet_zero<T><<<blocks_for(nb), BLOCK, 0, st>>>(L, y);
    if (n_partial) *n_partial = gi + blocks_for(L.n_shared);
    return hipGetLastError();
}
template hipError_t launch_tensor<double>(const LevelView<double> &, int, int, const double *, const double *,
                                          double *, double *, int *, hipStream_t);
template hipError_t launch_tensor<float>(const LevelView<float> &, int, int, const float *, const float *, float *,
                                         double *, int *, hipStream_t);

int tensor_partial_count(int n, int n_tet, int n_shared)
{
    int n_seg = 0;
    const dim3 g = stored_grid(n, n_tet, n_seg);
    return (int)(g.x * g.y) + blocks_for(n_shared);
}

hipError_t launch_form_diag(const LevelView<double> &L, int form, int mask, double *diag, double *partial,
                            int *n_partial, hipStream_t st)
{
    int gi = 0;
    if (form <= 1) {
        int n_seg = 0;
        const dim3 g = stored_grid(L.n, L.n_tet, n_seg);
        gi = (int)(g.x * g.y);
        if (g.x) {
            if (form == 0) k_form_diag<0><<<g, BLOCK, 0, st>>>(L, diag, partial, n_seg);
            else k_form_diag<1><<<g, BLOCK, 0, st>>>(L, diag, partial, n_seg);
        }
    } else if (form == 2) {
        int n_seg = 0;
        const dim3 g = stored_grid(L.n, L.n_tet, n_seg);
        gi = (int)(g.x * g.y);
        if (g.x) k_form_diag<2><<<g, BLOCK, 0, st>>>(L, diag, partial, n_seg);
    }
    const int gs = blocks_for(L.n_shared);
    const double *coef = form == 0 ? L.sh_ct : form == 1 ? L.sh_ctn : L.sh_cn;
    const int width = form <= 1 ? L.sh_wt : L.sh_w;
    if (gs) k_shared_diag<<<gs, BLOCK, 0, st>>>(L, coef, width, form == 3 ? mask : 0, diag, partial + gi);
    *n_partial = gi + gs;
    return hipGetLastError();
}

template hipError_t launch_store_stencils<double>(const LevelView<double> &, double *, hipStream_t);
template hipError_t launch_store_stencils<float>(const LevelView<double> &, float *, hipStream_t);

// ---------------------------------------------------------------- coarse solve
// u[copies of row r] = sum_c Ainv[r][c] f[gather[c]] in FP64 (u zeroed
// before): one wave per row, lanes stride over the columns (coalesced row
// reads), wave-wide sum
// the coarse right-hand side gathered once (one slot per coarse unknown) in FP64
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_coarse_gather(const int64_t *__restrict__ gather, const T *__restrict__ f,
                                                          double *__restrict__ fc, int nu)
{
    const int c = blockIdx.x * BLOCK + threadIdx.x;
    if (c < nu) fc[c] = (double)f[gather[c]];
}

// u = A^-1 f on the coarse level: one wave per row (four per block), the row
// streamed against the gathered right-hand side with two independent sums
// per lane, the result written to every copy of the node
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_coarse(const double *__restrict__ ainv, int nu,
                                                  const double *__restrict__ fc,
                                                  const int32_t *__restrict__ coff,
                                                  const int64_t *__restrict__ cslot, T *__restrict__ u)
{
    const int r = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= nu) return;  // whole wave
    const double *row = ainv + (int64_t)r * nu;
    double a0 = 0.0, a1 = 0.0;
    int c = lane;
    for (; c + 64 < nu; c += 128) {
        a0 += row[c] * fc[c];
        a1 += row[c + 64] * fc[c + 64];
    }
    if (c < nu) a0 += row[c] * fc[c];
    double acc = a0 + a1;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0)
        for (int p = coff[r]; p < coff[r + 1]; ++p) u[cslot[p]] = (T)acc;
}

template <typename T>
hipError_t launch_coarse_solve(const double *ainv, int nu, const int64_t *gather,
                               const int32_t *copy_off, const int64_t *copy_slot, const T *f, T *u,
                               double *fc, hipStream_t st)
{
    if (nu <= 0) return hipSuccess;
    k_coarse_gather<T><<<blocks_for(nu), BLOCK, 0, st>>>(gather, f, fc, nu);
    k_coarse<T><<<(nu + BLOCK / 64 - 1) / (BLOCK / 64), BLOCK, 0, st>>>(ainv, nu, fc, copy_off, copy_slot, u);
    return hipGetLastError();
}

// Dense inverse on the device by Gauss-Jordan elimination with partial
// pivoting on the augmented n x 2n matrix M = [A | I] (row-major, FP64).
// Step c: the pivot row p (largest |M[r][c]|, r >= c; the first on ties) and
// its value; swap rows c and p while scaling the new row c by 1/pivot; copy
// column c; subtract f_r x row c from every other row r (columns c..2n-1:
// left of c every row already holds 0 in A's part).  flag[0] is set when a
// pivot is 0 (singular matrix).
__global__ __launch_bounds__(BLOCK) void k_gj_pivot(const double *__restrict__ M, int n, int c,
                                                   int *__restrict__ piv, double *__restrict__ pval,
                                                   int *__restrict__ flag)
{
    __shared__ double bv[BLOCK];
    __shared__ int bi[BLOCK];
    const int64_t w = 2 * (int64_t)n;
    double best = -1.0;
    int bidx = n;
    for (int r = c + threadIdx.x; r < n; r += BLOCK) {
        const double v = fabs(M[(int64_t)r * w + c]);
        if (v > best) { best = v; bidx = r; }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    for (int h = BLOCK / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            const double v2 = bv[threadIdx.x + h];
            const int i2 = bi[threadIdx.x + h];
            if (v2 > bv[threadIdx.x] || (v2 == bv[threadIdx.x] && i2 < bi[threadIdx.x])) {
                bv[threadIdx.x] = v2;
                bi[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int p = bi[0] < n ? bi[0] : c;
        const double v = M[(int64_t)p * w + c];
        piv[0] = p;
        pval[0] = v;
        if (!(fabs(v) > 0.0)) flag[0] = 1;
    }
}

__global__ __launch_bounds__(BLOCK) void k_gj_swap_scale(double *__restrict__ M, int n, int c,
                                                        const int *__restrict__ piv,
                                                        const double *__restrict__ pval)
{
    const int64_t w = 2 * (int64_t)n;
    const int64_t k = c + (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= w) return;
    const int p = piv[0];
    const double v = pval[0];
    const double a = M[(int64_t)c * w + k], b = M[(int64_t)p * w + k];
    M[(int64_t)c * w + k] = b / v;
    if (p != c) M[(int64_t)p * w + k] = a;
}

__global__ __launch_bounds__(BLOCK) void k_gj_column(const double *__restrict__ M, int n, int c,
                                                    double *__restrict__ fcol)
{
    const int r = blockIdx.x * BLOCK + threadIdx.x;
    if (r < n) fcol[r] = r == c ? 0.0 : M[(int64_t)r * 2 * n + c];
}

__global__ __launch_bounds__(BLOCK) void k_gj_eliminate(double *__restrict__ M, int n, int c,
                                                       const double *__restrict__ fcol)
{
    const int64_t w = 2 * (int64_t)n;
    const int64_t k = c + (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int r = blockIdx.y;
    if (k >= w || r == c) return;
    const double f = fcol[r];
    if (f != 0.0) M[(int64_t)r * w + k] -= f * M[(int64_t)c * w + k];
}

__global__ __launch_bounds__(BLOCK) void k_gj_extract(const double *__restrict__ M, int n, double *__restrict__ ainv)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q >= (int64_t)n * n) return;
    const int64_t r = q / n, col = q - r * n;
    ainv[q] = M[r * 2 * n + n + col];
}

// work: n * 2n doubles holding [A | I] on entry; ainv: n * n; scratch: 2
// ints and n + 1 doubles (pivot row and value, column copy)
hipError_t launch_dense_inverse(double *work, int n, double *ainv, int *iscr, double *dscr, hipStream_t st)
{
    if (n <= 0 || n > 65535) return hipErrorInvalidValue;
    const int64_t w = 2 * (int64_t)n;
    for (int c = 0; c < n; ++c) {
        const unsigned gx = (unsigned)((w - c + BLOCK - 1) / BLOCK);
        k_gj_pivot<<<1, BLOCK, 0, st>>>(work, n, c, iscr, dscr, iscr + 1);
        k_gj_swap_scale<<<gx, BLOCK, 0, st>>>(work, n, c, iscr, dscr);
        k_gj_column<<<blocks_for(n), BLOCK, 0, st>>>(work, n, c, dscr + 1);
        k_gj_eliminate<<<dim3(gx, (unsigned)n), BLOCK, 0, st>>>(work, n, c, dscr + 1);
    }
    k_gj_extract<<<blocks_for((int64_t)n * n), BLOCK, 0, st>>>(work, n, ainv);
    return hipGetLastError();
}

// ---------------------------------------------------------------- misc
template <typename T>
__global__ void k_fill(T *x, T v, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n) x[q] = v;
}
template <typename T>
hipError_t launch_fill(T *x, T v, int64_t n, hipStream_t st)
{
    if (n > 0) k_fill<T><<<blocks_for(n), BLOCK, 0, st>>>(x, v, n);
    return hipGetLastError();
}

template <typename Ti, typename To>
__global__ void k_convert(const Ti *__restrict__ in, To *__restrict__ out, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n) out[q] = (To)in[q];
}
template <typename Ti, typename To>
hipError_t launch_convert(const Ti *in, To *out, int64_t n, hipStream_t st)
{
    k_convert<Ti, To><<<blocks_for(n), BLOCK, 0, st>>>(in, out, n);
    return hipGetLastError();
}

__global__ void k_add_f32(double *__restrict__ u, const float *__restrict__ c, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n) u[q] += (double)c[q];
}
hipError_t launch_add_f32_to_f64(double *u, const float *c, int64_t n, hipStream_t st)
{
    k_add_f32<<<blocks_for(n), BLOCK, 0, st>>>(u, c, n);
    return hipGetLastError();
}

// coarse nodes are the fine nodes with doubled lattice coordinates
template <typename T>
__global__ void k_inject(const T *__restrict__ kf, int nf, T *__restrict__ kc, int nc, int n_tet,
                         int64_t Spad_f, int64_t Spad_c)
{
    const int S = tc32(nc);
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q >= (int64_t)S * n_tet) return;
    const int tet = (int)(q / S), s = (int)(q - (int64_t)tet * S);
    int i, j, k;
    decode_slot(nc, s, i, j, k);
    kc[tet * Spad_c + s] = kf[tet * Spad_f + slot32(nf, 2 * i, 2 * j, 2 * k)];
}
template <typename T>
hipError_t launch_inject(const T *kf, int nf, T *kc, int nc, int n_tet, int64_t Spad_f,
                         int64_t Spad_c, hipStream_t st)
{
    k_inject<T><<<blocks_for((int64_t)tet_count(nc) * n_tet), BLOCK, 0, st>>>(kf, nf, kc, nc, n_tet,
                                                                             Spad_f, Spad_c);
    return hipGetLastError();
}

// Coarse coefficients as geometric full-weighting averages of the next finer
// level's: k_c = exp(sum_f P_fc log k_f / sum_f P_fc), P the P1
// interpolation (P_fc = 1 for the coincident fine node, 1/2 for the midpoint
// of each coarse edge at c).  Macro-tet interior nodes: the coincident node
// and the 14 edge midpoints of the same tet (total weight 8).  Nodes on macro
// faces, edges and vertices (Dirichlet ones included): from a list of their
// distinct fine support nodes over all copies, written to every copy.
__global__ __launch_bounds__(BLOCK) void k_coarsen_volume(const double *__restrict__ kf, int nf,
                                                         double *__restrict__ kc, int nc, int64_t Spad_f,
                                                         int64_t Spad_c)
{
    int i, j, k, s;
    if (!plane_point(nc, i, j, k, s)) return;
    if (i == 0 || j == 0 || k == 0 || i + j + k == nc) return;
    const int tet = blockIdx.z;
    const double *__restrict__ fb = kf + (int64_t)tet * Spad_f;
    const int sf = slot32(nf, 2 * i, 2 * j, 2 * k);
    int nb[NDIR];
    neighbour_slots(sf, 2 * (i + j), nf - 2 * k, nb);
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < NDIR; ++d) acc += log(fb[nb[d]]);
    kc[(int64_t)tet * Spad_c + s] = exp((log(fb[sf]) + 0.5 * acc) / 8.0);
}

__global__ __launch_bounds__(BLOCK) void k_coarsen_list(const double *__restrict__ kf, double *__restrict__ kc,
                                                       int n_nodes, const int32_t *__restrict__ off,
                                                       const int64_t *__restrict__ fslot,
                                                       const double *__restrict__ w,
                                                       const int32_t *__restrict__ coff,
                                                       const int64_t *__restrict__ cslot)
{
    const int q = blockIdx.x * BLOCK + threadIdx.x;
    if (q >= n_nodes) return;
    double acc = 0.0, ws = 0.0;
    for (int e = off[q]; e < off[q + 1]; ++e) {
        acc += w[e] * log(kf[fslot[e]]);
        ws += w[e];
    }
    const double v = exp(acc / ws);
    for (int c = coff[q]; c < coff[q + 1]; ++c) kc[cslot[c]] = v;
}

hipError_t launch_coarsen(const double *kf, int nf, double *kc, int nc, int n_tet, int64_t Spad_f, int64_t Spad_c,
                          int n_list, const int32_t *off, const int64_t *fslot, const double *w,
                          const int32_t *coff, const int64_t *cslot, hipStream_t st)
{
    if (nc >= 4) k_coarsen_volume<<<plane_grid(nc, n_tet), BLOCK, 0, st>>>(kf, nf, kc, nc, Spad_f, Spad_c);
    if (n_list) k_coarsen_list<<<blocks_for(n_list), BLOCK, 0, st>>>(kf, kc, n_list, off, fslot, w, coff, cslot);
    return hipGetLastError();
}

// map[q] = canonical node of slot q, or -(node+1) on a Dirichlet slot (then 0
// is written unless keep_dirichlet); padding slots are not touched
template <typename T>
__global__ void k_from_canon(const T *__restrict__ canon, const int32_t *__restrict__ map,
                             T *__restrict__ slots, int64_t n, int keep_dirichlet, int S,
                             int64_t Spad)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q >= n || q % Spad >= S) return;
    const int32_t c = map[q];
    slots[q] = c >= 0 ? canon[c] : (keep_dirichlet ? canon[-c - 1] : T(0));
}
template <typename T>
hipError_t launch_from_canonical(const T *canon, const int32_t *slot2canon, T *slots, int64_t n,
                                 int keep_dirichlet, int S, int64_t Spad, hipStream_t st)
{
    k_from_canon<T><<<blocks_for(n), BLOCK, 0, st>>>(canon, slot2canon, slots, n, keep_dirichlet, S,
                                                     Spad);
    return hipGetLastError();
}

template <typename T>
__global__ void k_to_canon(const T *__restrict__ slots, const int64_t *__restrict__ map,
                           T *__restrict__ canon, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n) canon[q] = slots[map[q]];
}
template <typename T>
hipError_t launch_to_canonical(const T *slots, const int64_t *canon2slot, T *canon, int64_t n,
                               hipStream_t st)
{
    k_to_canon<T><<<blocks_for(n), BLOCK, 0, st>>>(slots, canon2slot, canon, n);
    return hipGetLastError();
}

__global__ void k_positive(const double *__restrict__ k, int64_t n, int *bad)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n && !(k[q] > 0.0 && k[q] < 1e300)) atomicOr(bad, 1);
}
hipError_t launch_positive_check(const double *k, int64_t n, int *bad, hipStream_t st)
{
    k_positive<<<blocks_for(n), BLOCK, 0, st>>>(k, n, bad);
    return hipGetLastError();
}

// ---------------------------------------------------------------- instantiations
#define HHG_INST(T)                                                                               \
    template hipError_t launch_scaled<T>(const LevelView<T> &, int, const T *, const T *, T *,     \
                                         double *, int *, hipStream_t);                            \
    template hipError_t launch_nodal<T>(const LevelView<T> &, const T *, T *, hipStream_t);        \
    template hipError_t launch_correction<T>(const LevelView<T> &, const CorrView<T> &, int,       \
                                             const T *, T *, double *, hipStream_t);               \
    template hipError_t launch_stored<T>(const LevelView<T> &, const CorrView<T> &, const T *, const T *, \
                                         T *, hipStream_t);                                        \
    template hipError_t launch_cheb_sweep_mixed<T>(const LevelView<T> &, const CorrView<T> &, int,      \
                                                   const T *, const T *, T *, const ChebArgs<T> &,      \
                                                   hipStream_t);                                        \
    template hipError_t launch_scalar_form<T>(const LevelView<T> &, const CorrView<T> &, int, int, int,   \
                                              const T *, const T *, T *, double *, int *, hipStream_t); \
    template hipError_t launch_mixed<T>(const LevelView<T> &, const CorrView<T> &, const T *, T *, int, \
                                        hipStream_t);                                              \
    template hipError_t launch_cheb_sweep<T>(const LevelView<T> &, const CorrView<T> &, const T *, \
                                             const T *, T *, const ChebArgs<T> &, hipStream_t);    \
    template hipError_t launch_diag<T>(const LevelView<T> &, T *, double *, double *, double *,    \
                                       int *, hipStream_t);                                        \
    template hipError_t launch_invert_diag<T>(T *, int64_t, hipStream_t);                          \
    template hipError_t launch_jacobi_update<T>(T *, const T *, const T *, T, int64_t,             \
                                                hipStream_t);                                      \
    template hipError_t launch_cheb_update<T>(T *, T *, const T *, const T *, T, T, int64_t,       \
                                              hipStream_t);                                        \
    template hipError_t launch_restrict<T>(const LevelView<T> &, const LevelView<T> &, const T *,  \
                                           T *, hipStream_t);                                      \
    template hipError_t launch_prolong_add<T>(const LevelView<T> &, const LevelView<T> &,          \
                                              const T *, T *, hipStream_t);                        \
    template hipError_t launch_coarse_solve<T>(const double *, int, const int64_t *,               \
                                               const int32_t *, const int64_t *, const T *, T *,   \
                                               double *, hipStream_t);                             \
    template hipError_t launch_fill<T>(T *, T, int64_t, hipStream_t);                              \
    template hipError_t launch_inject<T>(const T *, int, T *, int, int, int64_t, int64_t,          \
                                         hipStream_t);                                             \
    template hipError_t launch_from_canonical<T>(const T *, const int32_t *, T *, int64_t, int,    \
                                                 int, int64_t, hipStream_t);                       \
    template hipError_t launch_to_canonical<T>(const T *, const int64_t *, T *, int64_t,           \
                                               hipStream_t);

HHG_INST(double)
HHG_INST(float)
template hipError_t launch_convert<double, float>(const double *, float *, int64_t, hipStream_t);
template hipError_t launch_convert<float, double>(const float *, double *, int64_t, hipStream_t);

}  // namespace hhg
