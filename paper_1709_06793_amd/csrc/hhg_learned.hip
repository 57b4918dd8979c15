// hhg_learned.hip -- kernels of the learned smoothing correction: features from
// the 15-point neighbourhood, a 32 -> 16 -> 16 -> 1 ReLU network with BF16
// weights on the matrix cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation),
// its parameter gradient, and the smoothing update that uses it.
//
// Features of an interior node i (positions p = 0: the node, p = 1..14: the
// lattice neighbours in DIR order):  s = max_p |r_p| + 1e-30,
// x_p = r_p * (1/s) (the reciprocal and each product rounded to FP32), x_{15+p} = L_p - L_0
// (L = log k rounded to FP32), x_30 = x_31 = 0.
// Network:  h1 = bf16(relu(W1 bf16(x) + b1)),  h2 = relu(W2 h1 + b2),
// c = w3 . h2 + b3.  Nodes on macro faces/edges/vertices and Dirichlet nodes
// get c = 0.
//
// Matrix-core mapping: for 16 nodes at a time the wave forms the transposed
// products C1^T = W1 X^T (two K=16 steps) and C2^T = W2 H1^T.  In the 16x16x16
// layout lane l holds A[l%16][4(l/16)+q], B[4(l/16)+q][l%16] and
// D[4(l/16)+q][l%16] (q = 0..3), so the output of layer 1 is already the B
// operand of layer 2 and no data moves between the layers.
#include <hip/hip_runtime.h>

#include "hhg_internal.h"
#include "hhg_lattice.h"
#include "hhg_learned.h"
#include "hhg_march.h"

namespace hhg {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int ltc32(int m) { return (m + 1) * (m + 2) * (m + 3) / 6; }

__device__ __forceinline__ void ldecode(int n, int s, int &i, int &j, int &k)
{
    const int q = ltc32(n) - s;
    int m = (int)(cbrtf(6.0f * (float)q)) - 2;
    m = m < 0 ? 0 : m;
    while (ltc32(m) < q) ++m;
    while (m > 0 && ltc32(m - 1) >= q) --m;
    k = n - m;
    const int t = s - (ltc32(n) - ltc32(m));
    int d = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while ((d + 1) * (d + 2) / 2 <= t) ++d;
    while (d > 0 && d * (d + 1) / 2 > t) --d;
    i = t - d * (d + 1) / 2;
    j = d - i;
}

// slot offsets of the 14 neighbours (DIR order) of slot s = (i,j,k), sd = i+j, m = n-k
__device__ __forceinline__ void lneighbours(int s, int sd, int m, int nb[NDIR])
{
    const int up = s + (m + 1) * (m + 2) / 2, dn = s - (m + 2) * (m + 3) / 2;
    nb[0] = s + sd + 2; nb[1] = s + sd + 1; nb[2] = up; nb[3] = s + 1;
    nb[4] = dn + sd + 2; nb[5] = dn + sd + 1; nb[6] = up + 1;
    nb[7] = s - sd - 1; nb[8] = s - sd; nb[9] = dn; nb[10] = s - 1;
    nb[11] = up - sd - 1; nb[12] = up - sd; nb[13] = dn - 1;
}

// round-to-nearest-even float -> bf16 bits
__device__ __forceinline__ unsigned short to_bf16(float f)
{
    const unsigned int u = __float_as_uint(f);
    const unsigned int r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }
// two floats to packed bf16 bits (low = a) with the hardware conversion
// (round to nearest, ties to even: the same bits as to_bf16 for finite values)
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned int pack_bf16(float a, float b)
{
    const f32x2 v = {a, b};
    const bf16x2v h = __builtin_convertvector(v, bf16x2v);
    unsigned int u;
    __builtin_memcpy(&u, &h, 4);
    return u;
}

// max(x, 0) as one integer max on the bit pattern: a negative float is a
// negative integer, so every finite x maps to its ReLU (-0 to +0)
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// features of slot s (interior node assumed): 32 values and the scale
__device__ __forceinline__ void node_features(const LevelView<float> &L, const float *__restrict__ r,
                                              const float *__restrict__ logk, int64_t base, int s,
                                              int sd, int k, float x[LN_IN], float &scale)
{
    int nb[NDIR];
    lneighbours(s, sd, L.n - k, nb);
    float rp[15], lp[15];
    rp[0] = r[base + s];
    lp[0] = logk[base + s];
#pragma unroll
    for (int d = 0; d < NDIR; ++d) {
        rp[d + 1] = r[base + nb[d]];
        lp[d + 1] = logk[base + nb[d]];
    }
    float m = 0.0f;
#pragma unroll
    for (int p = 0; p < 15; ++p) m = fmaxf(m, fabsf(rp[p]));
    scale = m + 1e-30f;
    const float inv = 1.0f / scale;
#pragma unroll
    for (int p = 0; p < 15; ++p) {
        x[p] = rp[p] * inv;
        x[15 + p] = lp[p] - lp[0];
    }
    x[30] = 0.0f;
    x[31] = 0.0f;
}

// ---------------------------------------------------------------- forward (MFMA)
// c[slot] = network output, sc[slot] = s * c, s_out[slot] = s (each nullable).
// Column marching, the traversal of the operator's interior kernel: a wave takes 64 consecutive in-plane offsets (lanes 1..62
// hold nodes) and walks a chunk of planes with the planes of r and log k in
// rotating registers (three coalesced loads per array and plane, neighbours
// at i+-1 from the adjacent lanes).  Per plane each lane forms its node's
// features, the wave stages them in LDS as BF16 and evaluates the network
// for its 64 lanes in four groups of 16 on the matrix cores.  Extra blocks
// write 0 to every slot on the tet's boundary.
// With u given (the learned smoothing step), the kernel also applies
// u <- u + D^{-1}(omega r + s c) at every slot of the lattice (c = 0 on the
// tet's boundary slots), so no separate update pass runs.
__global__ __launch_bounds__(BLOCK) void k_learned_fwd_march(LevelView<float> L, const float *__restrict__ r,
                                                             const float *__restrict__ logk,
                                                             const unsigned short *__restrict__ wbf,
                                                             float *__restrict__ c_out,
                                                             float *__restrict__ sc_out,
                                                             float *__restrict__ s_out,
                                                             float *__restrict__ u,
                                                             const float *__restrict__ invd, float omega)
{
    constexpr int NS = 4;
    // bf16 features of a lane's node: 16 words, rows 18 words apart (the
    // operand reads of 16 rows then fall in distinct banks)
    constexpr int XW = 18;
    __shared__ unsigned int xs[BLOCK * XW];
    __shared__ float cs[BLOCK];
    const int per_tet = L.vpt + L.bpt2;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    if (lb >= L.n_tet * per_tet) return;
    const int tet = lb / per_tet;
    int b;
    const bool marching = march_block(lb - tet * per_tet, L.vpt, L.bpt2, b);
    const int64_t base = (int64_t)tet * L.Spad;
    if (!marching) {
        const int e = b * BLOCK + threadIdx.x;
        if (e < L.n_bnd) {
            const int64_t sl = base + (L.bnd[e] >> 4);
            if (c_out) c_out[sl] = 0.0f;
            if (sc_out) sc_out[sl] = 0.0f;
            if (s_out) s_out[sl] = 0.0f;
            if (u) u[sl] += invd[sl] * (omega * r[sl] + 0.0f);
        }
        return;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int item = __builtin_amdgcn_readfirstlane(b * 4 + wave);
    if (item >= L.n_items) return;
    const uint2 it = L.items[item];
    const int n = L.n;
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
    const int lastk = row_lane ? min(n - 1 - sd, k1) : -1;
    const int64_t bytes = (int64_t)L.S * 4;
    const __amdgpu_buffer_rsrc_t rr = tet_rsrc(r + base, bytes);
    const __amdgpu_buffer_rsrc_t rl = tet_rsrc(logk + base, bytes);
    // a missing output gets an empty range: every store to it is dropped
    const __amdgpu_buffer_rsrc_t rc = tet_rsrc(c_out ? c_out + base : r + base, c_out ? bytes : 0);
    const __amdgpu_buffer_rsrc_t rsc = tet_rsrc(sc_out ? sc_out + base : r + base, sc_out ? bytes : 0);
    const __amdgpu_buffer_rsrc_t rs = tet_rsrc(s_out ? s_out + base : r + base, s_out ? bytes : 0);
    const __amdgpu_buffer_rsrc_t ru = tet_rsrc(u ? u + base : r + base, u ? bytes : 0);
    const __amdgpu_buffer_rsrc_t rid = tet_rsrc(u ? invd + base : r + base, u ? bytes : 0);
    const int vo[3] = {t >= 0 ? t - sd : 0, t >= 0 ? t : 0, t >= 0 ? t + sd + 1 : 0};
    const int Sn = tc32(n);
    auto plane = [&](int p) { return Sn - tc32(n - p); };
    // per-lane weight operands (A of the three products, biases, w3)
    const int row = lane & 15, kq = 4 * (lane >> 4);
    bf16x4 a1lo, a1hi, a2;
    for (int q = 0; q < 4; ++q) {
        a1lo[q] = (short)wbf[row * 32 + kq + q];
        a1hi[q] = (short)wbf[row * 32 + 16 + kq + q];
        a2[q] = (short)wbf[528 + row * 16 + kq + q];
    }
    float b1v[4], b2v[4], w3v[4];
    for (int q = 0; q < 4; ++q) {
        b1v[q] = from_bf16(wbf[512 + kq + q]);
        b2v[q] = from_bf16(wbf[784 + kq + q]);
        w3v[q] = from_bf16(wbf[800 + kq + q]);
    }
    const float b3 = from_bf16(wbf[816]);
    MPlane<float> R[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        mplane_load<float, MODE_APPLY>(R[q], rr, rl, rr, vo, plane(k0 - 1 + q));
        __builtin_amdgcn_sched_barrier(0);
    }
    mplane_shift_mid(R[0]);
    mplane_shift_up(R[1]);
    constexpr int DROP = 0x7ffffff0;
    for (int kb = k0; kb <= k1; kb += NS) {
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int k = kb + q;
            MPlane<float> &M = R[q % NS], &C = R[(q + 1) % NS], &P = R[(q + 2) % NS];
            const bool live = k <= lastk;
            const int so = live ? (plane(k) + vo[1]) * 4 : DROP;
            // the node's iterate and inverse diagonal, issued before the
            // feature and network work that hides their latency (an empty
            // range reads 0 when there is no update)
            const float u_old = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ru, so, 0, 0));
            const float id = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rid, so, 0, 0));
            mplane_shift_mid(C);
            mplane_shift_up(P);
            // node first, then the neighbours in DIR order
            const float rp[15] = {C.u[1], C.u_sp_r, C.u[2], P.u[1], C.u_s_r, M.u_sp_r, M.u[2], P.u_s_r,
                                  C.u_sm_l, C.u[0], M.u[1], C.u_s_l, P.u_sm_l, P.u[0], M.u_s_l};
            const float lp[15] = {C.k[1], C.k_sp_r, C.k[2], P.k[1], C.k_s_r, M.k_sp_r, M.k[2], P.k_s_r,
                                  C.k_sm_l, C.k[0], M.k[1], C.k_s_l, P.k_sm_l, P.k[0], M.k_s_l};
            float mx = 0.0f;
#pragma unroll
            for (int p2 = 0; p2 < 15; ++p2) mx = fmaxf(mx, fabsf(rp[p2]));
            const float scale = mx + 1e-30f;
            const float inv = 1.0f / scale;
            float x[32];
#pragma unroll
            for (int p2 = 0; p2 < 15; ++p2) {
                x[p2] = rp[p2] * inv;
                x[15 + p2] = lp[p2] - lp[0];
            }
            x[30] = 0.0f;
            x[31] = 0.0f;
            uint2 *mine = reinterpret_cast<uint2 *>(xs + threadIdx.x * XW);
#pragma unroll
            for (int w2 = 0; w2 < 8; ++w2)
                mine[w2] = make_uint2(pack_bf16(x[4 * w2], x[4 * w2 + 1]), pack_bf16(x[4 * w2 + 2], x[4 * w2 + 3]));
            __builtin_amdgcn_wave_barrier();
            // the four groups of 16 nodes interleaved (operand reads, then
            // each layer's products for all groups, then the reductions), so
            // that no product or cross-lane exchange waits for its own
            // predecessor alone; the biases start the accumulators (one FP32
            // sum of the products and the bias, as the reference's single
            // rounding bounds it)
            bf16x4 xlo[4], xhi[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const uint2 *src = reinterpret_cast<const uint2 *>(xs + (wave * 64 + g * 16 + row) * XW);
                const uint2 lo = src[lane >> 4], hi = src[4 + (lane >> 4)];
                __builtin_memcpy(&xlo[g], &lo, 8);
                __builtin_memcpy(&xhi[g], &hi, 8);
            }
            f32x4 acc[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                acc[g] = f32x4{b1v[0], b1v[1], b1v[2], b1v[3]};
                acc[g] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1lo, xlo[g], acc[g], 0, 0, 0);
            }
#pragma unroll
            for (int g = 0; g < 4; ++g) acc[g] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1hi, xhi[g], acc[g], 0, 0, 0);
            f32x4 acc2[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const uint2 hp = make_uint2(pack_bf16(relu(acc[g][0]), relu(acc[g][1])),
                                            pack_bf16(relu(acc[g][2]), relu(acc[g][3])));
                bf16x4 h1;
                __builtin_memcpy(&h1, &hp, 8);
                acc2[g] = f32x4{b2v[0], b2v[1], b2v[2], b2v[3]};
                acc2[g] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, h1, acc2[g], 0, 0, 0);
            }
            float part[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                part[g] = 0.0f;
                for (int q2 = 0; q2 < 4; ++q2) part[g] += w3v[q2] * relu(acc2[g][q2]);
            }
#pragma unroll
            for (int g = 0; g < 4; ++g) part[g] += __shfl_xor(part[g], 16, 64);
#pragma unroll
            for (int g = 0; g < 4; ++g) part[g] += __shfl_xor(part[g], 32, 64);
            if (lane < 16) {
#pragma unroll
                for (int g = 0; g < 4; ++g) cs[wave * 64 + g * 16 + lane] = part[g] + b3;
            }
            __builtin_amdgcn_wave_barrier();
            const float c = cs[threadIdx.x];
            const float scv = c * scale;
            bstore(c, rc, so);
            bstore(scv, rsc, so);
            bstore(scale, rs, so);
            bstore(u_old + id * (omega * rp[0] + scv), ru, so);
            mplane_load<float, MODE_APPLY>(M, rr, rl, rr, vo, plane(k - 1 + NS));
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

static int fwd_grid(const LevelView<float> &L)
{
    const int nb = L.n_tet * (L.vpt + L.bpt2);
    return ((nb + 7) / 8) * 8;
}

template <>
hipError_t launch_learned_forward<float>(const LevelView<float> &L, const LearnedState &S,
                                         const float *r, const float *logk, float *c, hipStream_t st)
{
    k_learned_fwd_march<<<fwd_grid(L), BLOCK, 0, st>>>(L, r, logk, S.wbf, c, nullptr, nullptr, nullptr, nullptr,
                                                        0.0f);
    return hipGetLastError();
}

hipError_t launch_learned_step(const LevelView<float> &L, const LearnedState &S, const float *r, const float *logk,
                               float *u, const float *invd, float omega, hipStream_t st)
{
    k_learned_fwd_march<<<fwd_grid(L), BLOCK, 0, st>>>(L, r, logk, S.wbf, nullptr, nullptr, nullptr, u, invd, omega);
    return hipGetLastError();
}

hipError_t launch_learned_forward_full(const LevelView<float> &L, const LearnedState &S,
                                       const float *r, const float *logk, float *c, float *sc,
                                       float *s, hipStream_t st)
{
    k_learned_fwd_march<<<fwd_grid(L), BLOCK, 0, st>>>(L, r, logk, S.wbf, c, sc, s, nullptr, nullptr, 0.0f);
    return hipGetLastError();
}

// ---------------------------------------------------------------- backward (FP32)
// Per block of LBW nodes: recompute the forward in FP32 (same bf16 roundings),
// back-propagate g, and sum the per-node outer products over the block into
// one partial gradient (817 floats) per block; a second kernel adds the
// partials in block order.
constexpr int LBW = 128;
constexpr int LROW = 32 + 16 + 16 + 16 + 16 + 1;  // x, h1, dz1, dz2, h2, g per node

__global__ __launch_bounds__(LBW) void k_learned_bwd(LevelView<float> L, const float *__restrict__ r,
                                                     const float *__restrict__ logk,
                                                     const unsigned short *__restrict__ wbf,
                                                     const float *__restrict__ gvec,
                                                     float *__restrict__ gpart)
{
    __shared__ float buf[LBW][LROW + 1];
    const int per_tet = (L.S + LBW - 1) / LBW;
    const int tet = blockIdx.x / per_tet;
    const int s = (blockIdx.x - tet * per_tet) * LBW + threadIdx.x;
    const int64_t base = (int64_t)tet * L.Spad;
    float *me = buf[threadIdx.x];
    bool interior = false;
    int i = 0, j = 0, k = 0;
    if (tet < L.n_tet && s < L.S) {
        ldecode(L.n, s, i, j, k);
        interior = i > 0 && j > 0 && k > 0 && i + j + k < L.n;
    }
    if (interior) {
        float x[LN_IN], scale;
        node_features(L, r, logk, base, s, i + j, k, x, scale);
        for (int f = 0; f < LN_IN; ++f) x[f] = from_bf16(to_bf16(x[f]));
        float h1[16], z1p[16], h2[16], z2p[16];
        for (int h = 0; h < 16; ++h) {
            float a = 0.0f;
            for (int f = 0; f < LN_IN; ++f) a += from_bf16(wbf[h * 32 + f]) * x[f];
            const float z = a + from_bf16(wbf[512 + h]);
            z1p[h] = z > 0.0f ? 1.0f : 0.0f;
            h1[h] = from_bf16(to_bf16(fmaxf(z, 0.0f)));
        }
        for (int h = 0; h < 16; ++h) {
            float a = 0.0f;
            for (int q = 0; q < 16; ++q) a += from_bf16(wbf[528 + h * 16 + q]) * h1[q];
            const float z = a + from_bf16(wbf[784 + h]);
            z2p[h] = z > 0.0f ? 1.0f : 0.0f;
            h2[h] = fmaxf(z, 0.0f);
        }
        const float g = gvec[base + s];
        float dz2[16], dz1[16];
        for (int h = 0; h < 16; ++h) dz2[h] = g * from_bf16(wbf[800 + h]) * z2p[h];
        for (int q = 0; q < 16; ++q) {
            float a = 0.0f;
            for (int h = 0; h < 16; ++h) a += from_bf16(wbf[528 + h * 16 + q]) * dz2[h];
            dz1[q] = a * z1p[q];
        }
        for (int f = 0; f < 32; ++f) me[f] = x[f];
        for (int h = 0; h < 16; ++h) {
            me[32 + h] = h1[h];
            me[48 + h] = dz1[h];
            me[64 + h] = dz2[h];
            me[80 + h] = h2[h];
        }
        me[96] = g;
    } else {
        for (int q = 0; q < LROW; ++q) me[q] = 0.0f;
    }
    __syncthreads();
    // parameter p of the block partial: sum over the block's nodes
    float *out = gpart + (int64_t)blockIdx.x * LN_NPARAM;
    for (int p = threadIdx.x; p < LN_NPARAM; p += LBW) {
        float a = 0.0f;
        if (p < 512) {            // dW1[h][f] = dz1[h] x[f]
            const int h = p >> 5, f = p & 31;
            for (int q = 0; q < LBW; ++q) a += buf[q][48 + h] * buf[q][f];
        } else if (p < 528) {     // db1
            for (int q = 0; q < LBW; ++q) a += buf[q][48 + p - 512];
        } else if (p < 784) {     // dW2[h][q'] = dz2[h] h1[q']
            const int h = (p - 528) >> 4, q2 = (p - 528) & 15;
            for (int q = 0; q < LBW; ++q) a += buf[q][64 + h] * buf[q][32 + q2];
        } else if (p < 800) {     // db2
            for (int q = 0; q < LBW; ++q) a += buf[q][64 + p - 784];
        } else if (p < 816) {     // dw3 = g h2
            for (int q = 0; q < LBW; ++q) a += buf[q][96] * buf[q][80 + p - 800];
        } else {                  // db3
            for (int q = 0; q < LBW; ++q) a += buf[q][96];
        }
        out[p] = a;
    }
}

__global__ void k_learned_gred(const float *__restrict__ gpart, int nblk, float *__restrict__ g)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= LN_NPARAM) return;
    double a = 0.0;
    for (int b = 0; b < nblk; ++b) a += (double)gpart[(int64_t)b * LN_NPARAM + p];
    g[p] = (float)a;
}

int learned_bwd_blocks(const LevelView<float> &L) { return L.n_tet * ((L.S + LBW - 1) / LBW); }

hipError_t launch_learned_backward(const LevelView<float> &L, const LearnedState &S, const float *r,
                                   const float *logk, const float *g, hipStream_t st)
{
    const int nb = learned_bwd_blocks(L);
    k_learned_bwd<<<nb, LBW, 0, st>>>(L, r, logk, S.wbf, g, S.gpart);
    k_learned_gred<<<(LN_NPARAM + 255) / 256, 256, 0, st>>>(S.gpart, nb, S.dgrad);
    return hipGetLastError();
}

// training: e1 = e - D^{-1}(omega r + s c)
__global__ void k_learned_err(const float *__restrict__ e, const float *__restrict__ r,
                              const float *__restrict__ sc, const float *__restrict__ invd,
                              float omega, float *__restrict__ e1, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n) e1[q] = e[q] - invd[q] * (omega * r[q] + sc[q]);
}
hipError_t launch_learned_err(const float *e, const float *r, const float *sc, const float *invd,
                              float omega, float *e1, int64_t n, hipStream_t st)
{
    k_learned_err<<<(int)((n + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(e, r, sc, invd, omega, e1, n);
    return hipGetLastError();
}

// training: g = -2 (A e1) s D^{-1} / E0 on nodes with a network output
__global__ void k_learned_lossgrad(const float *__restrict__ ae1, const float *__restrict__ s,
                                   const float *__restrict__ invd, double inv_e0,
                                   float *__restrict__ g, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n) g[q] = (float)(-2.0 * (double)ae1[q] * (double)s[q] * (double)invd[q] * inv_e0);
}
hipError_t launch_learned_lossgrad(const float *ae1, const float *s, const float *invd, double inv_e0,
                                   float *g, int64_t n, hipStream_t st)
{
    k_learned_lossgrad<<<(int)((n + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(ae1, s, invd, inv_e0, g, n);
    return hipGetLastError();
}

// weighted dot product sum_q w_q a_q b_q (w = 1 on one copy of every unknown)
__global__ __launch_bounds__(BLOCK) void k_dot_owned(const float *__restrict__ a, const float *__restrict__ b,
                                                     const uint8_t *__restrict__ own, int64_t n,
                                                     double *__restrict__ partial)
{
    __shared__ double red[BLOCK / 64];
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double v = (q < n && own[q]) ? (double)a[q] * (double)b[q] : 0.0;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < BLOCK / 64; ++w) v += red[w];
        partial[blockIdx.x] = v;
    }
}
hipError_t launch_dot_owned(const float *a, const float *b, const uint8_t *own, int64_t n,
                            double *partial, int *nblk, hipStream_t st)
{
    *nblk = (int)((n + BLOCK - 1) / BLOCK);
    k_dot_owned<<<*nblk, BLOCK, 0, st>>>(a, b, own, n, partial);
    return hipGetLastError();
}

// log k rounded to FP32 (log in FP64)
__global__ void k_logk(const double *__restrict__ k, float *__restrict__ lk, int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n) lk[q] = (float)log(k[q]);
}
hipError_t launch_logk(const double *k, float *lk, int64_t n, hipStream_t st)
{
    k_logk<<<(int)((n + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(k, lk, n);
    return hipGetLastError();
}

// FP32 master weights -> BF16 bits
__global__ void k_to_bf16(const float *__restrict__ w, unsigned short *__restrict__ wb, int n)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) wb[q] = to_bf16(w[q]);
}
hipError_t launch_weights_bf16(const float *w, unsigned short *wb, int n, hipStream_t st)
{
    k_to_bf16<<<(n + 255) / 256, 256, 0, st>>>(w, wb, n);
    return hipGetLastError();
}

// training pair: r = (float) r64, e = (float)(u* - u)
__global__ void k_pair(const double *__restrict__ r64, const double *__restrict__ us,
                       const double *__restrict__ u, float *__restrict__ r, float *__restrict__ e,
                       int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (q < n) {
        r[q] = (float)r64[q];
        e[q] = (float)(us[q] - u[q]);
    }
}
hipError_t launch_pair(const double *r64, const double *us, const double *u, float *r, float *e,
                       int64_t n, hipStream_t st)
{
    k_pair<<<(int)((n + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(r64, us, u, r, e, n);
    return hipGetLastError();
}

}  // namespace hhg
